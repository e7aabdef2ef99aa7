// Double-distribution (f, g) fused pull stream-collide kernel, D2Q9, ideal gas.
//
// One launch advances one time step of Eq. (LBM_f) and Eq. (LBM_g) of Sec. II C in the order
// of Fig. 1, with an optional uniform body force F and heat source Q (float32/float64 storage):
//   pull f_i, g_i from x - c_i (periodic in x; periodic or half-way bounce-back walls in y);
//   rho = sum f, rho u = sum c f + F/2, rho E = sum g + (u.F + Q)/2;  T = (E - u^2/2)/c_v,
//   P = rho R T, theta = P/rho (ideal gas, Sec. III A);
//   Galilean correction Phi_aa = -(1/rho) d_a(rho u_a^3 + 3 rho u_a (theta - 1/3)) with a
//   finite-difference derivative of the moments of the neighbouring nodes at the same time
//   level (central, or one-sided on the upwind side of u_a);
//   shifted state u* = u + F/rho, theta* = theta + (gamma - 1) Q/rho,
//   T* = T + Q/(rho c_v) - F.F/(2 rho^2 c_v) (u*, theta*, T* = u, theta, T without sources);
//   f^eq, f* = rho prod_a Psi(u*_a, theta* + u*_a^2 + Phi_aa), g^eq, g* = g^eq(rho, u*, T*,
//   theta*) (closed form of the operator-generated energy equilibrium; q^c = 0 at Prandtl
//   number 1);
//   beta = 1/(2 tau + 1), tau = mu/P, omega = 2 beta;
//   f~ = f + omega (f^eq - f) + (1 - beta)(f* - f^eq),
//   g~ = g + omega (g^eq - g) + (1 - beta)(g* - g^eq).
//
// Tiling. A workgroup of 256 threads owns 256 - 2 HALO columns (256 - 2 HALO - 2 with staged
// rows, whose outermost thread on each side only stages) and `rows` rows; each thread holds
// one column (the HALO columns at either side only supply neighbour moments) and walks the
// rows y0 - HALO .. y0 + rows + HALO - 1 bottom to top. For each row it gathers the
// populations, computes the moments and the correction fluxes phi_a, exchanges phi_x across the
// row through LDS (x derivative) and keeps phi_y of the last 2 HALO + 1 rows of its own column
// in LDS (y derivative). A row is collided HALO rows after it was gathered, when the y
// stencil is complete; its populations wait in a register ring of HALO + 1 slots. Each
// population of the lattice is read once from HBM by its owning workgroup; halo rows and
// columns are re-read by the neighbouring workgroup (L2 hits for the x halo of neighbouring
// tiles on the same XCD).
//
// Storage policies (IO template parameter):
//   IoFull<S>    float32 or float64 planes holding f_i - w_i and g_i - v_i, where w, v are the
//                equilibria at rest at the reference state rho = 1, T = 1;
//   IoRed<Codec> float32 moments (rho - 1, u_x, u_y, T - 1) + 16-bit non-equilibrium part, 6 of
//                the 9 f values and 8 of the 9 g values (see reduced_common.h); every row of
//                the window is rebuilt once per workgroup into LDS (software-pipelined: the raw
//                values of the row after next are loaded while the current row collides) and
//                the pull reads the rebuilt populations from there.
// The register ring holds the pulled populations shifted by (w, v) in the policy's ring type.
// Arithmetic is float64.
#include "ddf_common.h"
#include "reduced_common.h"

#include <cstdlib>
#include <type_traits>

namespace lbm {

template <typename S>
struct IoFull {
  using ring_t = S;
  static constexpr bool kStaged = false;
  static constexpr int kEdge = 0;
  static constexpr int kStageFloats = 1;
  const S* A;
  S* B;
  int64_t plane;
  const S* nb;  // boundary rows of the non-equilibrium extrapolation walls (k_ddf_neq_rows)
  struct RawRow {};
  __device__ __forceinline__ void fetch_row(RawRow&, int, int, int, int, int64_t, int) const {}
  __device__ __forceinline__ void put_row(float*, const RawRow&, int, int, int, const DdfParams&) const {}
  __device__ __forceinline__ void gather(bool pull, int64_t r0, int64_t rm, int64_t rp, int x,
                                         int xm, int xp, bool top, bool bot, const DdfParams&,
                                         int, int, const float*, S (&hf)[9], S (&hg)[9]) const {
    if (pull) {
      gather9(A, plane, r0, rm, rp, x, xm, xp, top, bot, hf);
      gather9(A + 9 * plane, plane, r0, rm, rp, x, xm, xp, top, bot, hg);
    } else {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        hf[i] = A[i * plane + r0 + x];
        hg[i] = A[(9 + i) * plane + r0 + x];
      }
    }
  }
  // pre-collision populations of boundary row `side` (0: y = 0, 1: y = ny - 1), column x
  __device__ __forceinline__ void gather_wall(int side, int x, int64_t pitch, S (&hf)[9],
                                             S (&hg)[9]) const {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      hf[i] = nb[(side * 18 + i) * pitch + x];
      hg[i] = nb[(side * 18 + 9 + i) * pitch + x];
    }
  }
  __device__ __forceinline__ void store(int64_t off, int i, double htf, double, double htg,
                                        double) const {
    store_nt(B + i * plane + off, (S)htf);
    store_nt(B + (9 + i) * plane + off, (S)htg);
  }
  __device__ __forceinline__ void store_moments(int64_t, const double*, double) const {}
};

template <typename Codec>
struct IoRed {
  using ring_t = float;
  const float* M;     // 4 moment planes
  const uint16_t* N;  // kRedF f planes, then kRedG g planes
  float* Mo;
  uint16_t* No;
  int64_t plane;
  float s_enc, s_dec;
  // post-collision population ii of node `src`, rebuilt and shifted by the rest state
  __device__ __forceinline__ void pop(int64_t src, int ii, const DdfParams& p, double& hf,
                                      double& hg) const {
    const double rho = 1.0 + (double)M[src];
    const double ux = (double)M[plane + src];
    const double uy = (double)M[2 * plane + src];
    const double T = 1.0 + (double)M[3 * plane + src];
    const double theta = p.R * T, e = p.cv * T;
    double pa, ca, pb, cb;
    axis_eq1(ii % 3 - 1, ux, theta, pa, ca);
    axis_eq1(ii / 3 - 1, uy, theta, pb, cb);
    const double fe = rho * pa * pb;
    const double ge = rho * (e * pa * pb + ca * pb + pa * cb);
    hf = fe + neq_f<Codec>(N, plane, src, ii, s_dec) - p.wf[ii];
    hg = ge + neq_g<Codec>(N + kRedF * plane, plane, src, ii, s_dec) - p.wg[ii];
  }
  // Staging: the rows of the 3-row pull window are decoded once per workgroup into LDS,
  // stage[slot][c][k] with c = thread index, column x_first + c (one column per thread, so no
  // wavefront decodes twice; the outermost thread on each side only stages) and k = 0..8
  // f - w, 9..17 g - v (19 floats per column: an odd stride keeps the lanes on distinct LDS
  // banks).
  static constexpr bool kStaged = true;
  static constexpr int kEdge = 1;  // threads per side that stage but do not pull
  static constexpr int kCols = kBlock, kStride = 19;
  static constexpr int kStageFloats = 3 * kCols * kStride;
  // Raw stored values of one column: 4 moments, 6 f codes, 8 g codes.
  struct Raw {
    float m[4];
    uint16_t n[kRedF + kRedG];
  };
  using RawRow = Raw;
  __device__ __forceinline__ void fetch(Raw& v, int rr, int c, int nx, int64_t pitch) const {
    const int xg = ((c % nx) + nx) % nx;
    const int64_t off = (int64_t)rr * pitch + xg;
#pragma unroll
    for (int k = 0; k < 4; ++k) v.m[k] = M[k * plane + off];
#pragma unroll
    for (int k = 0; k < kRedF + kRedG; ++k) v.n[k] = N[k * plane + off];
  }
  __device__ __forceinline__ void decode(const Raw& v, float* dst, const DdfParams& p) const {
    const double rho = 1.0 + (double)v.m[0];
    const double ux = (double)v.m[1];
    const double uy = (double)v.m[2];
    const double T = 1.0 + (double)v.m[3];
    double nf[9], ng[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      if (f_slot(i) >= 0) nf[i] = (double)Codec::dec(v.n[f_slot(i)], s_dec);
      if (g_slot(i) >= 0) ng[i] = (double)Codec::dec(v.n[kRedF + g_slot(i)], s_dec);
    }
    nf[5] = nf[0] - nf[2] + nf[3] + nf[6] - nf[8];
    nf[7] = nf[0] + nf[1] + nf[2] - nf[6] - nf[8];
    nf[4] = -(((nf[0] + nf[1]) + (nf[2] + nf[3])) + ((nf[5] + nf[6]) + (nf[7] + nf[8])));
    ng[4] = -(((ng[0] + ng[1]) + (ng[2] + ng[3])) + ((ng[5] + ng[6]) + (ng[7] + ng[8])));
    double fe[9], ge[9];
    equilibria(rho, ux, uy, p.R * T, p.cv * T, fe, ge);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      dst[i] = (float)(fe[i] - p.wf[i] + nf[i]);
      dst[9 + i] = (float)(ge[i] - p.wg[i] + ng[i]);
    }
  }
  // rows beyond a wall are never pulled (bounce-back) and are not staged
  __device__ __forceinline__ void fetch_row(RawRow& rw, int r, int ny, int nx, int x_first,
                                            int64_t pitch, int walls) const {
    if (walls && (r < 0 || r >= ny)) return;
    const int rr = ((r % ny) + ny) % ny;
    fetch(rw, rr, x_first + (int)threadIdx.x, nx, pitch);
  }
  __device__ __forceinline__ void put_row(float* st, const RawRow& rw, int r, int ny, int walls,
                                          const DdfParams& p) const {
    if (walls && (r < 0 || r >= ny)) return;
    float* dst = st + ((r % 3) + 3) % 3 * (kCols * kStride);
    decode(rw, dst + threadIdx.x * kStride, p);
  }
  // pull of node (staged column tid, row r) from LDS; 1 <= tid <= kBlock - 2
  __device__ __forceinline__ void gather(bool pull, int64_t, int64_t, int64_t, int, int, int,
                                         bool top, bool bot, const DdfParams&, int r, int tid,
                                         const float* st, float (&hf)[9], float (&hg)[9]) const {
    auto at = [&](int row, int c, int k) {
      return st[((row % 3) + 3) % 3 * (kCols * kStride) + c * kStride + k];
    };
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int ka = i % 3, kb = i / 3;
      const bool bounce = (kb == 2 && bot) || (kb == 0 && top);
      if (!pull) {
        hf[i] = at(r, tid, i);
        hg[i] = at(r, tid, 9 + i);
      } else if (bounce) {
        hf[i] = at(r, tid, 8 - i);
        hg[i] = at(r, tid, 17 - i);
      } else {
        hf[i] = at(r - (kb - 1), tid - (ka - 1), i);
        hg[i] = at(r - (kb - 1), tid - (ka - 1), 9 + i);
      }
    }
  }
  __device__ __forceinline__ void store(int64_t off, int i, double htf, double hfe, double htg,
                                        double hge) const {
    if (f_slot(i) >= 0) store_nt(No + f_slot(i) * plane + off, Codec::enc((float)(htf - hfe), s_enc));
    if (g_slot(i) >= 0) store_nt(No + (kRedF + g_slot(i)) * plane + off, Codec::enc((float)(htg - hge), s_enc));
  }
  __device__ __forceinline__ void store_moments(int64_t off, const double* m, double inv_R) const {
    store_nt(Mo + off, (float)(m[0] - 1.0));
    store_nt(Mo + plane + off, (float)m[1]);
    store_nt(Mo + 2 * plane + off, (float)m[2]);
    store_nt(Mo + 3 * plane + off, (float)(m[3] * inv_R - 1.0));
  }
};

// WALLS: 0 = periodic in y, 1 = bounce-back walls, 2 = non-equilibrium extrapolation walls
// (boundary rows rebuilt by k_ddf_neq_rows into io.nb).
// EXT: 0 = paper's collision without sources, 1 = extended path (sources and/or transport
// control, ideal gas), 2 = extended path for the van der Waals fluid.
template <class IO, int HALO, int WALLS, bool PULL, bool DIAG, int EXT>
__global__ void __launch_bounds__(kBlock)
k_ddf_d2q9(IO io, int nx, int ny, int64_t pitch, DdfParams prm, int rows,
           double* __restrict__ partials) {
  using S = typename IO::ring_t;
  constexpr int H1 = HALO + 1;
  constexpr int P = 2 * HALO + 1;
  constexpr int EDGE = IO::kEdge;  // staging-only threads per side
  constexpr int TXI = kBlock - 2 * HALO - 2 * EDGE;
  __shared__ double s_phix[2][kBlock];
  __shared__ double s_phiy[P][kBlock];
  __shared__ float s_stage[IO::kStageFloats];
  // extended path with transport control: T and u_x of the gathered row (x derivatives) and T,
  // u_y of the last P rows per column (y derivatives)
  constexpr bool X = EXT > 0;
  constexpr bool VDW = EXT == 2;
  constexpr int NE = X ? kBlock : 1;
  constexpr int NH = VDW ? kBlock : 1;
  __shared__ double s_tx[2][NE], s_ux[2][NE], s_hx[2][NH];
  __shared__ double s_ty[P][NE], s_uy[P][NE], s_hy[P][NH];
  constexpr int NM = X ? (VDW ? 9 : 8) : 6;

  const int nbx = gridDim.x;
  // per-XCD contiguous tiles for float32/float64 storage; the staged reduced-storage variant
  // measured 1.6% faster in hardware order
  const int hw = blockIdx.x + nbx * blockIdx.y;
  const int tile = IO::kStaged ? hw : xcd_tile(hw, nbx * gridDim.y);
  const int bx = tile % nbx;
  const int by = tile / nbx;
  const int tid = threadIdx.x;
  const int x0 = bx * TXI;
  const int xu = x0 - HALO - EDGE + tid;          // unwrapped column
  const int x = ((xu % nx) + nx) % nx;            // periodic in x
  const bool own = tid >= HALO + EDGE && tid < kBlock - HALO - EDGE && xu < nx;
  const bool puller = tid >= EDGE && tid < kBlock - EDGE;  // has all its pull sources
  const int xm = x == 0 ? nx - 1 : x - 1;
  const int xp = x == nx - 1 ? 0 : x + 1;
  const int y0 = by * rows;
  const int yend = min(y0 + rows, ny);
  const int count = (yend - y0) + 2 * HALO;       // window rows


  S ring_f[H1][9], ring_g[H1][9];
  double ring_m[H1][NM];  // rho, u_x, u_y, theta, e, Phi_xx [, dT/dx, du_x/dx, dh/dx]
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};

  // Staged rows are software-pipelined: the raw values of row r + 2 are fetched into registers
  // while row r is processed and decoded into LDS at the start of the next iteration.
  const int x_first = x0 - HALO - EDGE;  // first staged column (thread 0's)
  typename IO::RawRow raw;
  if (IO::kStaged) {
    io.fetch_row(raw, y0 - HALO - 1, ny, nx, x_first, pitch, WALLS);
    io.put_row(s_stage, raw, y0 - HALO - 1, ny, WALLS, prm);
    io.fetch_row(raw, y0 - HALO, ny, nx, x_first, pitch, WALLS);
    io.put_row(s_stage, raw, y0 - HALO, ny, WALLS, prm);
    io.fetch_row(raw, y0 - HALO + 1, ny, nx, x_first, pitch, WALLS);
  }
  // Pull of window row r (periodic in y unless walls) into hf, hg.
  auto gather_row = [&](int r, S(&hf)[9], S(&hg)[9]) {
    const int rr = WALLS ? r : ((r % ny) + ny) % ny;
    const int ym = rr == 0 ? ny - 1 : rr - 1;
    const int yp = rr == ny - 1 ? 0 : rr + 1;
    const int64_t r0 = (int64_t)rr * pitch, rm = (int64_t)ym * pitch, rp = (int64_t)yp * pitch;
    const bool top = WALLS && rr == ny - 1, bot = WALLS && rr == 0;
    if constexpr (WALLS == 2) {
      if (top || bot) {  // rebuilt boundary rows (k_ddf_neq_rows)
        io.gather_wall(top ? 1 : 0, x, pitch, hf, hg);
        return;
      }
    }
    io.gather(PULL, r0, rm, rp, x, xm, xp, top, bot, prm, r, tid, s_stage, hf, hg);
  };
  // window row w exists (inside the window and, with walls, inside the lattice)
  auto row_of = [&](int w) { return y0 - HALO + w; };
  auto real_row = [&](int w) {
    const int r = row_of(w);
    return w < count && (WALLS ? (r >= 0 && r < ny) : true);
  };
  for (int k = 0; k < count; k += H1) {
#pragma unroll
    for (int j = 0; j < H1; ++j) {
      const int w = k + j;                 // window index (block-uniform)
      const int r = row_of(w);             // row being gathered
      if (IO::kStaged) {
        // slot (r + 1) mod 3 holds row r - 2, last read by the gather of row r - 1, which is
        // ordered before this write by the barrier that follows that gather
        io.put_row(s_stage, raw, r + 1, ny, WALLS, prm);
        __syncthreads();
        io.fetch_row(raw, r + 2, ny, nx, x_first, pitch, WALLS);
      }
      const bool in_window = w < count;
      const bool row_real = real_row(w);
      double phx = 0.0, phy = 0.0;
      if (row_real && puller) {
        // ---- gather (pull) ----------------------------------------------------------------
        gather_row(r, ring_f[j], ring_g[j]);
        // ---- moments and closure ------------------------------------------------------------
        Moments m;
        moments_closure_dev<X, VDW>(ring_f[j], ring_g[j], prm, m, prm.Fx, prm.Fy, prm.Q);
        ring_m[j][0] = m.rho;
        ring_m[j][1] = m.ux;
        ring_m[j][2] = m.uy;
        ring_m[j][3] = m.theta;
        ring_m[j][4] = m.e;
        phx = m.rho * m.ux * (m.ux * m.ux + 3.0 * (m.theta - 1.0 / 3.0));
        phy = m.rho * m.uy * (m.uy * m.uy + 3.0 * (m.theta - 1.0 / 3.0));
        if (X && prm.full) {
          const double T = node_temperature<VDW>(prm, m.rho, m.e, m.theta);
          s_tx[w & 1][tid] = T;
          s_ux[w & 1][tid] = m.ux;
          s_ty[((r % P) + P) % P][tid] = T;
          s_uy[((r % P) + P) % P][tid] = m.uy;
          if constexpr (VDW) {  // specific enthalpy h = e + P / rho
            s_hx[w & 1][tid] = m.e + m.theta;
            s_hy[((r % P) + P) % P][tid] = m.e + m.theta;
          }
        }
      }
      s_phix[w & 1][tid] = phx;
      s_phiy[((r % P) + P) % P][tid] = phy;
      __syncthreads();
      // ---- x derivatives of T and u_x (transport control) --------------------------------------
      if (X && prm.full && row_real && own) {
        ring_m[j][6] = 0.5 * (s_tx[w & 1][tid + 1] - s_tx[w & 1][tid - 1]);
        ring_m[j][7] = 0.5 * (s_ux[w & 1][tid + 1] - s_ux[w & 1][tid - 1]);
        if constexpr (VDW) ring_m[j][NM - 1] = 0.5 * (s_hx[w & 1][tid + 1] - s_hx[w & 1][tid - 1]);
      }
      // ---- x derivative of phi_x on the gathered row -----------------------------------------
      if (row_real && own && prm.phi) {
        const double* px = s_phix[w & 1];
        double d;
        if (HALO == 1) {
          d = 0.5 * (px[tid + 1] - px[tid - 1]);
        } else {
          // the upwind side follows u_x, on the boundary rows of NEQ walls the wall's u_x
          double key = ring_m[j][1];
          if (WALLS == 2 && (r == 0 || r == ny - 1)) key = prm.uw[r == 0 ? 0 : 1][0];
          d = upwind_or_central(px[tid - 2], px[tid - 1], px[tid], px[tid + 1], px[tid + 2], key);
        }
        ring_m[j][5] = -d;  // -d(phi_x)/dx; divided by rho at the collision
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
          if (HALO == 1) {
            d = 0.5 * (q[3] - q[1]);
          } else {
            // on the boundary rows of NEQ walls the side follows the wall's normal velocity,
            // zero: the y derivative there is central
            double key = ring_m[sc][2];
            if (WALLS == 2 && (c == 0 || c == ny - 1)) key = prm.uw[c == 0 ? 0 : 1][1];
            d = upwind_or_central(q[0], q[1], q[2], q[3], q[4], key);
          }
          phyy = -d;
        }
        double phxx = 0.0;
        if (prm.phi) {  // Phi_aa = -(1/rho) d(phi_a)/da: one reciprocal for both axes
          const double inv_rho = 1.0 / ring_m[sc][0];
          phxx = ring_m[sc][5] * inv_rho;
          phyy *= inv_rho;
        }
        // y derivatives of T and u_y (transport control), central with zero-order wall ghosts
        double dTdy = 0.0, duydy = 0.0, dhdy = 0.0;
        if (X && prm.full) {
          int rm1 = c - 1, rp1 = c + 1;
          if (WALLS) {
            rm1 = rm1 < 0 ? 0 : rm1;
            rp1 = rp1 > ny - 1 ? ny - 1 : rp1;
          }
          const int sm = ((rm1 % P) + P) % P, sp = ((rp1 % P) + P) % P;
          dTdy = 0.5 * (s_ty[sp][tid] - s_ty[sm][tid]);
          duydy = 0.5 * (s_uy[sp][tid] - s_uy[sm][tid]);
          if constexpr (VDW) dhdy = 0.5 * (s_hy[sp][tid] - s_hy[sm][tid]);
        }
        const int64_t off = (int64_t)cc * pitch + x;
        collide_ddf<X, VDW>(ring_f[sc], ring_g[sc], ring_m[sc], phxx, phyy, dTdy, duydy, dhdy, prm,
                    [&](int i, double htf, double hfe, double htg, double hge) {
                      io.store(off, i, htf, hfe, htg, hge);
                    });
        io.store_moments(off, ring_m[sc], prm.inv_R);
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
  double theta = prm.R * T[n], e = prm.cv * T[n];
  if (prm.eos) {  // van der Waals: theta = P / rho, e = c_v T - a rho
    theta = prm.R * T[n] / (1.0 - prm.vb * rho[n]) - prm.va * rho[n];
    e -= prm.va * rho[n];
  }
  double fe[9], ge[9];
  equilibria(rho[n], u[n], u[nodes + n], theta, e, fe, ge);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    A[i * plane + off] = (S)(fe[i] - prm.wf[i]);
    A[(9 + i) * plane + off] = (S)(ge[i] - prm.wg[i]);
  }
}

// rho, u, T of the stored state. The collision conserves rho, rho u and rho E without sources;
// with sources the stored (post-collision) sums carry a whole step of F and Q, so the moments
// at the same time are those of the closure with the sources of that collision negated
// (prm.Fx, prm.Fy, prm.Q hold them).
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
  if (prm.eos) moments_closure<true, true>(f, g, prm, m, -prm.Fx, -prm.Fy, -prm.Q);
  else moments_closure<true, false>(f, g, prm, m, -prm.Fx, -prm.Fy, -prm.Q);
  rho[n] = m.rho;
  u[n] = m.ux;
  u[nodes + n] = m.uy;
  T[n] = prm.eos ? (m.e + prm.va * m.rho) / prm.cv : m.theta / prm.R;
  edens[n] = m.rho * (m.e + 0.5 * (m.ux * m.ux + m.uy * m.uy));
}

// Population plane i (f_i for i < Q, g_(i-Q) after) decoded to float64; D2Q9 and D3Q27 (the
// rows of all planes are consecutive at `pitch`).
template <typename S>
__global__ void k_decode_ddf(int Q, int i, const S* __restrict__ Ai, int nx, int64_t nodes,
                             int64_t pitch, DdfParams prm, double* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  out[n] = (double)Ai[off] + (i < Q ? prm.wf[i] : prm.wg[i - Q]);
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
Grid make_grid_ddf(const Layout& L, int halo, bool reduced) {
  Grid G;
  G.bx = kBlock;
  // own columns per workgroup: kBlock - 2 halo, less one staging-only thread per side when
  // the rows are staged (the kernel's TXI)
  const int txi = kBlock - 2 * halo - (reduced ? 2 : 0);
  G.nbx = (L.nx + txi - 1) / txi;
  // rows per workgroup from sweeps on MI355X at 4096^2 with walls (float32, central Phi:
  // 2 -> 588 us, 4 -> 553, 8 -> 580, 16 -> 599; float32, upwind Phi: 4 -> 646, 8 -> 596,
  // 16 -> 586; reduced bf16: 8 -> 676, 16 -> 602, 32 -> 604): short windows give more
  // workgroups in flight, taller ones amortise the halo rows (two per side for the upwind
  // stencil) and the staged kernel's 2-row staging halo
  G.rows = reduced ? 16 : (halo == 2 ? 16 : 4);
#ifdef LBM_TUNING_ENV
  if (const char* v = getenv("LBM_DDF_ROWS")) G.rows = atoi(v);
#endif
  fit_rows(G, L.ny);
  return G;
}

template <class IO, int HALO, int WALLS, bool PULL, int EXT>
static void ddf_launch_s(const IO& io, const Layout& L, const Grid& G, const DdfParams& prm,
                         double* partials, hipStream_t s) {
  dim3 grid(G.nbx, G.nby), block(kBlock);
  if (partials)
    k_ddf_d2q9<IO, HALO, WALLS, PULL, true, EXT><<<grid, block, 0, s>>>(io, L.nx, L.ny, L.pitch, prm, G.rows, partials);
  else
    k_ddf_d2q9<IO, HALO, WALLS, PULL, false, EXT><<<grid, block, 0, s>>>(io, L.nx, L.ny, L.pitch, prm, G.rows, nullptr);
}

// The extended path (sources, transport control) exists for float32/float64 storage only (the
// context rejects it with reduced storage, whose codec assumes a non-equilibrium part without
// mass and momentum).
template <class IO, int HALO, int WALLS, bool PULL>
static void ddf_launch(const IO& io, const Layout& L, const Grid& G, const DdfParams& prm,
                       double* partials, hipStream_t s) {
  if constexpr (!IO::kStaged) {
    if (prm.eos) {
      ddf_launch_s<IO, HALO, WALLS, PULL, 2>(io, L, G, prm, partials, s);
      return;
    }
    if (prm.ext()) {
      ddf_launch_s<IO, HALO, WALLS, PULL, 1>(io, L, G, prm, partials, s);
      return;
    }
  }
  ddf_launch_s<IO, HALO, WALLS, PULL, 0>(io, L, G, prm, partials, s);
}

template <class IO, int HALO>
static void ddf_launch_w(bool walls, bool pull, const IO& io, const Layout& L, const Grid& G,
                         const DdfParams& prm, double* partials, hipStream_t s) {
  if (walls) {
    if constexpr (!IO::kStaged) {  // NEQ walls: float32 / float64 storage only
      if (prm.neq) {
        if (pull) ddf_launch<IO, HALO, 2, true>(io, L, G, prm, partials, s);
        else ddf_launch<IO, HALO, 2, false>(io, L, G, prm, partials, s);
        return;
      }
    }
    if (pull) ddf_launch<IO, HALO, 1, true>(io, L, G, prm, partials, s);
    else ddf_launch<IO, HALO, 1, false>(io, L, G, prm, partials, s);
  } else {
    if (pull) ddf_launch<IO, HALO, 0, true>(io, L, G, prm, partials, s);
    else ddf_launch<IO, HALO, 0, false>(io, L, G, prm, partials, s);
  }
}

template <class IO>
static void ddf_launch_h(bool walls, bool pull, const IO& io, const Layout& L, const Grid& G,
                         const DdfParams& prm, double* partials, hipStream_t s) {
  if (prm.phi == 2) ddf_launch_w<IO, 2>(walls, pull, io, L, G, prm, partials, s);
  else ddf_launch_w<IO, 1>(walls, pull, io, L, G, prm, partials, s);
}

// reduced buffer: 4 float32 moment planes, then kRedF + kRedG uint16 planes
template <typename Codec>
static IoRed<Codec> make_red(const void* A, void* B, const Layout& L, float se, float sd) {
  IoRed<Codec> io;
  io.M = static_cast<const float*>(A);
  io.N = reinterpret_cast<const uint16_t*>(io.M + 4 * L.plane);
  io.Mo = static_cast<float*>(B);
  io.No = reinterpret_cast<uint16_t*>(io.Mo + 4 * L.plane);
  io.plane = L.plane;
  io.s_enc = se;
  io.s_dec = sd;
  return io;
}

// Non-equilibrium extrapolation walls (App. B): the pre-collision populations of the boundary
// rows B (y = 0, ny - 1, on the walls) are f^eq(rho_B, u_W, T_W) + f_N - f^eq(rho_N, u_N, T_N)
// with N the neighbouring row (1, ny - 2), pulled like any fluid row (PULL = false: its own
// slots), and rho_B the pressure-continued or the literal density (neq_wall_state); VDW: the
// van der Waals closure at N and at the wall. One thread per column, gridDim.y = 2 walls; the
// rows go to nb[(side*18 + k)*pitch + x], k < 9 f - w, k >= 9 g - v.
template <typename S, bool PULL, bool VDW>
__global__ void __launch_bounds__(kBlock)
k_ddf_neq_rows(const S* __restrict__ A, int nx, int ny, int64_t pitch, int64_t plane,
               DdfParams prm, S* __restrict__ nb) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  const int side = blockIdx.y;
  const int N = side ? ny - 2 : 1;
  const int xm = x == 0 ? nx - 1 : x - 1;
  const int xp = x == nx - 1 ? 0 : x + 1;
  S hf[9], hg[9];
  const int64_t r0 = (int64_t)N * pitch;
  if (PULL) {
    gather9(A, plane, r0, r0 - pitch, r0 + pitch, x, xm, xp, false, false, hf);
    gather9(A + 9 * plane, plane, r0, r0 - pitch, r0 + pitch, x, xm, xp, false, false, hg);
  } else {
    for (int i = 0; i < 9; ++i) {
      hf[i] = A[i * plane + r0 + x];
      hg[i] = A[(9 + i) * plane + r0 + x];
    }
  }
  double f[9], g[9];
  for (int i = 0; i < 9; ++i) {
    f[i] = (double)hf[i] + prm.wf[i];
    g[i] = (double)hg[i] + prm.wg[i];
  }
  Moments m;
  moments_closure<false, VDW>(f, g, prm, m);
  double feN[9], geN[9], feB[9], geB[9];
  equilibria(m.rho, m.ux, m.uy, m.theta, m.e, feN, geN);
  const double TN = node_temperature<VDW>(prm, m.rho, m.e, m.theta);
  double rhoB, thetaW, eW;
  neq_wall_state<VDW>(prm, side, m.rho, TN, m.rho * m.theta, rhoB, thetaW, eW);
  equilibria(rhoB, prm.uw[side][0], prm.uw[side][1], thetaW, eW, feB, geB);
  for (int i = 0; i < 9; ++i) {
    nb[(side * 18 + i) * pitch + x] = (S)(feB[i] + (f[i] - feN[i]) - prm.wf[i]);
    nb[(side * 18 + 9 + i) * pitch + x] = (S)(geB[i] + (g[i] - geN[i]) - prm.wg[i]);
  }
}

// Rows per workgroup of the extended collisions (sources, transport control, van der Waals):
// their longer per-row arithmetic favours taller windows than the plain step's. Measured at
// 4096^2 with walls, central Phi, float32 (4 / 6 / 8 / 10 rows): sources 618 / 589 / 582 /
// 583 us, Pr 0.71 646 / 613 / 601 / 599, van der Waals 719 / 673 / 649 / 644; the plain and NEQ
// steps keep their 4 (552 / 568 at 6 and 561 / 580).
constexpr int kDdfExtRows = 8;

hipError_t launch_ddf(int fmt, bool walls, bool pull, const void* A, void* B, const Layout& L,
                      const Grid& G0, const DdfParams& prm, float s_enc, float s_dec,
                      double* partials, void* nb, int* records, hipStream_t s) {
  if (prm.ext() && fmt >= 2) return hipErrorInvalidValue;  // no extended path with reduced storage
  Grid G = G0;
  if (fmt < 2 && (prm.ext() || prm.eos) && G.rows < kDdfExtRows) {
    G.rows = kDdfExtRows;
    fit_rows(G, L.ny);
  }
  if (records) *records = G.blocks();
  if (prm.neq) {
    if (fmt >= 2 || !walls || !nb || L.ny < 3 || prm.src) return hipErrorInvalidValue;
    dim3 grid((L.nx + kBlock - 1) / kBlock, 2);
    auto rows = [&](auto tag, auto pl, auto vdw) {
      using S = decltype(tag);
      k_ddf_neq_rows<S, decltype(pl)::value, decltype(vdw)::value><<<grid, kBlock, 0, s>>>(
          static_cast<const S*>(A), L.nx, L.ny, L.pitch, L.plane, prm, static_cast<S*>(nb));
    };
    auto by_flags = [&](auto tag) {
      if (pull) {
        if (prm.eos) rows(tag, std::true_type{}, std::true_type{});
        else rows(tag, std::true_type{}, std::false_type{});
      } else {
        if (prm.eos) rows(tag, std::false_type{}, std::true_type{});
        else rows(tag, std::false_type{}, std::false_type{});
      }
    };
    if (fmt == 0) by_flags(float{});
    else by_flags(double{});
  }
  if (fmt == 0) {
    IoFull<float> io{static_cast<const float*>(A), static_cast<float*>(B), L.plane,
                     static_cast<const float*>(nb)};
    ddf_launch_h(walls, pull, io, L, G, prm, partials, s);
  } else if (fmt == 1) {
    IoFull<double> io{static_cast<const double*>(A), static_cast<double*>(B), L.plane,
                      static_cast<const double*>(nb)};
    ddf_launch_h(walls, pull, io, L, G, prm, partials, s);
  } else if (fmt == 2) {
    ddf_launch_h(walls, pull, make_red<CodecBF16>(A, B, L, s_enc, s_dec), L, G, prm, partials, s);
  } else {
    ddf_launch_h(walls, pull, make_red<CodecFP16>(A, B, L, s_enc, s_dec), L, G, prm, partials, s);
  }
  return hipGetLastError();
}

// ---- reduced-storage initialisation and read-out ------------------------------------------------
__global__ void k_init_ddf_red(const double* __restrict__ rho, const double* __restrict__ u,
                               const double* __restrict__ T, float* __restrict__ M,
                               uint16_t* __restrict__ N, int nx, int64_t nodes, int64_t pitch,
                               int64_t plane) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  M[off] = (float)(rho[n] - 1.0);
  M[plane + off] = (float)u[n];
  M[2 * plane + off] = (float)u[nodes + n];
  M[3 * plane + off] = (float)(T[n] - 1.0);
  for (int k = 0; k < kRedF + kRedG; ++k) N[k * plane + off] = 0;
}

__global__ void k_moments_ddf_red(const float* __restrict__ M, int nx, int64_t nodes, int64_t pitch,
                                  int64_t plane, DdfParams prm, double* __restrict__ rho,
                                  double* __restrict__ u, double* __restrict__ T,
                                  double* __restrict__ edens) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  const double r = 1.0 + (double)M[off], ux = (double)M[plane + off], uy = (double)M[2 * plane + off];
  const double t = 1.0 + (double)M[3 * plane + off];
  rho[n] = r;
  u[n] = ux;
  u[nodes + n] = uy;
  T[n] = t;
  edens[n] = r * (prm.cv * t + 0.5 * (ux * ux + uy * uy));
}

template <typename Codec>
__global__ void k_decode_ddf_red(int i, IoRed<Codec> io, int nx, int64_t nodes, int64_t pitch,
                                 DdfParams prm, double* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  double hf, hg;
  io.pop(off, i % 9, prm, hf, hg);
  out[n] = i < 9 ? hf + prm.wf[i] : hg + prm.wg[i - 9];
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_ddf_rest_state(const DdfParams& prm, double* out, hipStream_t s) {
  k_ddf_rest_state<<<1, 1, 0, s>>>(prm, out);
  return hipGetLastError();
}

hipError_t launch_init_ddf(int kind, const double* rho, const double* u, const double* T,
                           void* A, const Layout& L, const DdfParams& prm, hipStream_t s) {
  if (kind >= 2) {
    float* M = static_cast<float*>(A);
    k_init_ddf_red<<<nblk(L.nodes()), kBlock, 0, s>>>(rho, u, T, M, reinterpret_cast<uint16_t*>(M + 4 * L.plane), L.nx, L.nodes(), L.pitch, L.plane);
  } else if (kind == 0)
    k_init_ddf<float><<<nblk(L.nodes()), kBlock, 0, s>>>(rho, u, T, static_cast<float*>(A), L.nx, L.ny, L.pitch, L.plane, prm);
  else
    k_init_ddf<double><<<nblk(L.nodes()), kBlock, 0, s>>>(rho, u, T, static_cast<double*>(A), L.nx, L.ny, L.pitch, L.plane, prm);
  return hipGetLastError();
}

hipError_t launch_moments_ddf(int kind, const void* A, const Layout& L, const DdfParams& prm,
                              double* rho, double* u, double* T, double* edens, hipStream_t s) {
  if (kind >= 2)
    k_moments_ddf_red<<<nblk(L.nodes()), kBlock, 0, s>>>(static_cast<const float*>(A), L.nx, L.nodes(), L.pitch, L.plane, prm, rho, u, T, edens);
  else if (kind == 0)
    k_moments_ddf<float><<<nblk(L.nodes()), kBlock, 0, s>>>(static_cast<const float*>(A), L.nx, L.ny, L.pitch, L.plane, prm, rho, u, T, edens);
  else
    k_moments_ddf<double><<<nblk(L.nodes()), kBlock, 0, s>>>(static_cast<const double*>(A), L.nx, L.ny, L.pitch, L.plane, prm, rho, u, T, edens);
  return hipGetLastError();
}

hipError_t launch_decode_ddf(int kind, int Q, int i, const void* A, const Layout& L,
                             const DdfParams& prm, float s_dec, double* out, hipStream_t s) {
  if (kind == 2)
    k_decode_ddf_red<CodecBF16><<<nblk(L.nodes()), kBlock, 0, s>>>(i, make_red<CodecBF16>(A, nullptr, L, 1.0f, s_dec), L.nx, L.nodes(), L.pitch, prm, out);
  else if (kind == 3)
    k_decode_ddf_red<CodecFP16><<<nblk(L.nodes()), kBlock, 0, s>>>(i, make_red<CodecFP16>(A, nullptr, L, 1.0f, s_dec), L.nx, L.nodes(), L.pitch, prm, out);
  else if (kind == 0)
    k_decode_ddf<float><<<nblk(L.nodes()), kBlock, 0, s>>>(Q, i, static_cast<const float*>(A) + (int64_t)i * L.plane, L.nx, L.nodes(), L.pitch, prm, out);
  else
    k_decode_ddf<double><<<nblk(L.nodes()), kBlock, 0, s>>>(Q, i, static_cast<const double*>(A) + (int64_t)i * L.plane, L.nx, L.nodes(), L.pitch, prm, out);
  return hipGetLastError();
}

}  // namespace lbm
