// Double-distribution (f, g) stream-collide step for D3Q27, float32 or float64 storage:
// Eq. (LBM_f) and Eq. (LBM_g) of Sec. II C in the order of Fig. 1, for the ideal gas or the
// van der Waals fluid (Sec. III C), with the optional body force, heat source and transport
// control of the D2Q9 kernel (ddf.hip).
//
// With the central derivative of Phi one launch per step, k_ddf3_fused (below), marches along z
// and computes the fluxes and the collision together (after k_ddf3_neq_rows with NEQ walls).
// With the upwind derivative, or without Phi, two launches per step (three with NEQ walls):
//   k_ddf3_neq_rows rebuilds the pre-collision populations of the boundary planes y = 0 and
//                   y = ny - 1 of the non-equilibrium extrapolation walls (App. B) into a side
//                   buffer;
//   k_ddf3_flux     pulls the 27 + 27 populations of every node, computes its moments and
//                   writes the Galilean-correction fluxes phi_a = rho u_a (u_a^2 + 3 (theta - 1/3))
//                   (and, with transport control, T and u; for the van der Waals fluid also the
//                   enthalpy) to fields in the storage type;
//   k_ddf3_collide  pulls the same populations again, recomputes the same moments, takes the
//                   finite-difference derivatives of the neighbours' fields (central, or the
//                   upwind-biased stencil for phi), collides and stores.
// The second pull re-reads what the first one read: 432 B of populations per node in float32
// are read twice, so the pair moves about 1.5x the algorithmic traffic of one fused sweep; the
// one-launch step avoids that with a plane ring (the upwind stencil would need two planes of
// ring and of halo each way).
//
// Storage: 54 planes, f_i - w_i (i < 27) then g_i - v_i, with w, v the equilibria at rest at
// rho = 1, T = 1; i = (cx+1) + 3(cy+1) + 9(cz+1), opposite 26 - i. Walls in y: half-way
// bounce-back or NEQ extrapolation; x and z periodic. Arithmetic is float64.
#include "ddf_common.h"

#include <cstdlib>
#include <type_traits>

namespace lbm {

struct Moments3 {
  double rho, u[3], theta, e;
};

// Pull of the 27 + 27 populations of node (x, y, z): h_i = A_i(x - c_i), or the node's own
// opposite population where x - c_i lies beyond a y wall; PULL = false reads the node's own
// slots (the collide-only pass at creation). ROW_UNIFORM: (y, z) is the same for every lane of
// the wavefront (the sweeps, one x row per workgroup row), so the source rows are addressed
// from scalar bases with 32-bit column offsets; otherwise (the NEQ boundary rebuild, one (x, z)
// node per lane) every lane forms its own addresses.
template <typename S, bool WALLS, bool PULL, bool ROW_UNIFORM>
__device__ __forceinline__ void gather27(const S* __restrict__ A, int64_t plane, int nx, int ny,
                                         int nz, int64_t pitch, int x, int y, int z,
                                         S (&hf)[27], S (&hg)[27]) {
  const int64_t self = ((int64_t)z * ny + y) * pitch + x;
  if (!PULL) {
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      hf[i] = A[i * plane + self];
      hg[i] = A[(27 + i) * plane + self];
    }
    return;
  }
  const int xc[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};  // x - c_x
  const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
  const int zs[3] = {z == nz - 1 ? 0 : z + 1, z, z == 0 ? nz - 1 : z - 1};
  if constexpr (!ROW_UNIFORM) {
    int64_t pl = plane;  // re-declared: see the row-uniform path below
    asm volatile("" : "+s"(pl));
#pragma unroll
    for (int i = 0; i < 27; ++i) {
      const int a = i % 3, b = (i / 3) % 3, c = i / 9;
      const bool bounce = WALLS && ((b == 2 && y == 0) || (b == 0 && y == ny - 1));
      if (bounce) {
        hf[i] = A[(26 - i) * pl + self];
        hg[i] = A[(53 - i) * pl + self];
      } else {
        const int64_t src = ((int64_t)zs[c] * ny + ys[b]) * pitch + xc[a];
        hf[i] = A[i * pl + src];
        hg[i] = A[(27 + i) * pl + src];
      }
    }
    return;
  }
  const uint32_t xs[3] = {fresh((uint32_t)sizeof(S) * xc[0]), fresh((uint32_t)sizeof(S) * xc[1]),
                          fresh((uint32_t)sizeof(S) * xc[2])};
  const int64_t row = ((int64_t)z * ny + y) * pitch;
  // plane strides re-declared here (an empty asm): otherwise the compiler keeps the 54 plane
  // offsets of the loop-invariant products in scalar registers across the row loop and spills
  // them to vector lanes
  int64_t pl = plane;
  asm volatile("" : "+s"(pl));
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int a = i % 3, b = (i / 3) % 3, c = i / 9;
    const bool bounce = WALLS && ((b == 2 && y == 0) || (b == 0 && y == ny - 1));
    if (bounce) {
      hf[i] = *at_byte(sbase(A + (26 - i) * pl + row), xs[1]);
      hg[i] = *at_byte(sbase(A + (53 - i) * pl + row), xs[1]);
    } else {
      const int64_t src = ((int64_t)zs[c] * ny + ys[b]) * pitch;
      hf[i] = *at_byte(sbase(A + i * pl + src), xs[a]);
      hg[i] = *at_byte(sbase(A + (27 + i) * pl + src), xs[a]);
    }
  }
}

// Pre-collision populations of node (x, y, z). WALLS: 0 periodic in y, 1 bounce-back walls,
// 2 non-equilibrium extrapolation walls, whose boundary planes y = 0 and y = ny - 1 come
// rebuilt from nb (k_ddf3_neq_rows: 2 sides x 54 populations, each nz x pitch elements).
template <typename S, int WALLS, bool PULL, bool ROW_UNIFORM>
__device__ __forceinline__ void node_pops(const S* __restrict__ A, const S* __restrict__ nb,
                                          int64_t plane, int nx, int ny, int nz, int64_t pitch,
                                          int x, int y, int z, S (&hf)[27], S (&hg)[27]) {
  if constexpr (WALLS == 2) {
    if (y == 0 || y == ny - 1) {
      const int64_t nbp = (int64_t)nz * pitch;
      const int64_t o = (int64_t)(y == 0 ? 0 : 54) * nbp + (int64_t)z * pitch + x;
#pragma unroll
      for (int i = 0; i < 27; ++i) {
        hf[i] = nb[o + i * nbp];
        hg[i] = nb[o + (27 + i) * nbp];
      }
      return;
    }
  }
  gather27<S, (WALLS != 0), PULL, ROW_UNIFORM>(A, plane, nx, ny, nz, pitch, x, y, z, hf, hg);
}

// rho = sum f, rho u = sum c f + sF/2, rho E = sum g + (u.sF + sQ)/2 (Sec. II C), then
// T = (E - u^2/2)/c_v and theta = R T; for the van der Waals fluid (EXT = 2)
// T = (E - u^2/2 + a rho)/c_v (Eq. lbm_temp) and theta = P/rho. (sF, sQ) as in moments_closure
// (ddf_common.h); EXT = 0 takes no sources. The sums run over the stored deviations
// h = f - w, g - v and add the rest totals sum w, sum v once (p.wsum_f, p.wsum_g); sum c w
// vanishes, w being even in every velocity component.
template <int EXT, typename S>
__device__ __forceinline__ void moments3(const S (&hf)[27], const S (&hg)[27], const DdfParams& p,
                                         Moments3& m, double sFx, double sFy, double sFz,
                                         double sQ) {
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, rE = 0.0;
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const double f = (double)hf[i];
    rho += f;
    const int c[3] = {i % 3 - 1, (i / 3) % 3 - 1, i / 9 - 1};
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (c[a]) j[a] += c[a] > 0 ? f : -f;
    rE += (double)hg[i];
  }
  rho += p.wsum_f;
  rE += p.wsum_g;
  if (EXT) {
    j[0] += 0.5 * sFx;
    j[1] += 0.5 * sFy;
    j[2] += 0.5 * sFz;
  }
  const double inv = 1.0 / rho;
  m.rho = rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) m.u[a] = j[a] * inv;
  if (EXT) rE += 0.5 * ((m.u[0] * sFx + m.u[1] * sFy + m.u[2] * sFz) + sQ);
  m.e = rE * inv - 0.5 * (m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2]);
  if constexpr (EXT == 2) {
    const double T = (m.e + p.va * rho) / p.cv;
    m.theta = p.R * T / (1.0 - p.vb * rho) - p.va * rho;
  } else {
    m.theta = p.r_cv * m.e;
  }
}

// f^eq and g^eq in product form (Sec. II C; the operator-generated g^eq in closed form,
// g_i = rho [e psi_x psi_y psi_z + chi_x psi_y psi_z + psi_x chi_y psi_z + psi_x psi_y chi_z]).
__device__ __forceinline__ void equilibria3(double rho, double e, int i, const Axis (&ax)[3],
                                            double& fe, double& ge) {
  const int a = i % 3, b = (i / 3) % 3, c = i / 9;
  const double px = ax[0].psi[a], py = ax[1].psi[b], pz = ax[2].psi[c];
  const double pp = px * py * pz;
  fe = rho * pp;
  ge = rho * (e * pp + ax[0].chi[a] * py * pz + px * ax[1].chi[b] * pz + px * py * ax[2].chi[c]);
}

// Collision of one node (see collide_ddf in ddf_common.h for the D2Q9 form): ph[a] = Phi_aa,
// gT[a] = dT/da and divu = div u (used only when p.full), gh[a] = dh/da of the enthalpy
// h = e + P/rho (van der Waals only); sink(i, f~ - w, g~ - v). EXT: 0 without sources and
// transport terms, 1 with them (ideal gas), 2 the van der Waals fluid (gamma - 1, alpha and
// q^c = P (grad h - (k/mu) grad T) per node). sink(k, value): post-collision population k,
// shifted (k < 27: f~_k - w_k, else g~_{k-27} - v_{k-27}).
// FULL = false drops the transport terms at compile time (callers without them).
template <int EXT, bool FULL = true, typename S, typename Sink>
__device__ __forceinline__ void collide3(const S (&hf)[27], const S (&hg)[27], const Moments3& m,
                                         const double (&ph)[3], const double (&gT)[3],
                                         const double (&gh)[3], double divu, const DdfParams& p,
                                         const double* wf, const double* wg, Sink&& sink) {
  const double rho = m.rho, theta = m.theta, e = m.e;
  const double P = rho * theta;
  Axis X[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) axis_eq(m.u[a], theta, X[a]);
  Axis XS[3] = {X[0], X[1], X[2]};
  double es = e, q[3] = {0.0, 0.0, 0.0};
  if (EXT) {
    const double inv = 1.0 / rho;
    const double Fa[3] = {p.Fx, p.Fy, p.Fz};
    double thetas;
    if constexpr (EXT == 2) {
      const double omb = 1.0 - p.vb * rho;
      const double T = (e + p.va * rho) / p.cv;
      const double cs2 = p.R * T / (omb * omb) - 2.0 * p.va * rho +
                         T * p.R * p.R / (p.cv * omb * omb);
      const double alpha = 5.0 / 3.0 - rho * cs2 / P - p.eta;  // (D+2)/D - rho c_s^2/P - eta/mu
      thetas = theta + p.R / (omb * p.cv) * p.Q * inv + alpha * theta * divu;
#pragma unroll
      for (int a = 0; a < 3; ++a) q[a] = P * (gh[a] - p.kmu * gT[a]);
    } else {
      thetas = theta + p.r_cv * p.Q * inv;
      if (FULL && p.full) {
        thetas += p.alpha * theta * divu;
#pragma unroll
        for (int a = 0; a < 3; ++a) q[a] = P * p.qc * gT[a];
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) axis_eq(m.u[a] + Fa[a] * inv, thetas, XS[a]);
    es = e + p.Q * inv - 0.5 * (p.Fx * p.Fx + p.Fy * p.Fy + p.Fz * p.Fz) * inv * inv;
  }
  // Psi(c; u*, theta* + u*^2 + Phi) = psi* + Phi * (1/2, -1, 1/2)
  double s[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s[a][0] = XS[a].psi[0] + 0.5 * ph[a];
    s[a][1] = XS[a].psi[1] - ph[a];
    s[a][2] = XS[a].psi[2] + 0.5 * ph[a];
  }
  const double omega = 2.0 * P / (2.0 * p.mu + P);  // 2 beta, beta = 1/(2 tau + 1), tau = mu/P
  const double keep = 1.0 - 0.5 * omega;            // 1 - beta
  // all f first, then all g (the same arithmetic per value): fewer values are live at once
  // than with f_i and g_i together
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int a = i % 3, b = (i / 3) % 3, c = i / 9;
    double fe, ge;
    equilibria3(rho, e, i, X, fe, ge);
    const double hfe = fe - wf[i];
    const double f = (double)hf[i];
    const double fs = rho * (s[0][a] * s[1][b] * s[2][c]);
    sink(i, f + omega * (hfe - f) + keep * (fs - fe));
  }
#pragma unroll
  for (int i = 0; i < 27; ++i) {
    const int a = i % 3, b = (i / 3) % 3, c = i / 9;
    double fe, ge;
    equilibria3(rho, e, i, X, fe, ge);
    const double hge = ge - wg[i];
    const double g = (double)hg[i];
    double gstar_minus_ge = 0.0;
    if (EXT) {
      double gs, fsx;
      equilibria3(rho, es, i, XS, fsx, gs);
      // c_i . q^c / 2 on the six velocities with |c_i| = 1
      const int ca = a - 1, cb = b - 1, cc = c - 1;
      if ((FULL || EXT == 2) && ca * ca + cb * cb + cc * cc == 1)
        gs += 0.5 * (ca * q[0] + cb * q[1] + cc * q[2]);
      gstar_minus_ge = gs - ge;
    }
    sink(27 + i, g + omega * (hge - g) + keep * gstar_minus_ge);
  }
}

// ---- kernels --------------------------------------------------------------------------------
// The rest-state shift of the 54 populations in LDS, read per use: as kernel parameters the 54
// doubles took 108 scalar registers for the whole kernel and spilled some 330 of them to vector
// lanes (about 700 extra vector instructions per node in the collision sweep). The offset z is
// 0 but re-declared per row, so the reads stay at their uses instead of being hoisted into
// registers (the moments need only the shift's totals, held in DdfParams). Taken, with
// scalar-base row addressing, by the collisions without sources, transport terms or NEQ walls
// (kLean below) and by the one-launch step: 256^3 central 2226 -> 2152 us, upwind 2678 -> 2466 us; the
// extended sweeps (one wave per SIMD, ~310 registers) measured 2-3% slower with it and the NEQ
// sweeps 1.5% slower, so they keep the parameter arrays and per-lane addresses.
struct RestShift {
  double w[54];
  __device__ __forceinline__ void fill(const DdfParams& p) {
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < 27; ++i) {
        w[i] = p.wf[i];
        w[27 + i] = p.wg[i];
      }
    }
    __syncthreads();
  }
  __device__ __forceinline__ const double* at_row() const {
    int z = 0;
    asm volatile("" : "+v"(z));
    return w + z;
  }
};

// Fields written by k_ddf3_flux (in the storage type S, each `plane` elements at the population
// offsets): 0..2 phi_x, phi_y, phi_z;  with transport control 3: T, 4..6: u_x, u_y, u_z; for the
// van der Waals fluid 7: h = e + P/rho.
// With float32 storage the moments already carry the populations' float32 rounding, so float32
// fields add an error of the same order and halve the field traffic of both sweeps.
template <typename S, int WALLS, bool PULL, int EXT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_ddf3_flux(const S* __restrict__ A, const S* __restrict__ nb, int nx, int ny, int nz,
            int64_t pitch, int64_t plane, DdfParams prm, int rows, S* __restrict__ fld) {
  // scalar-base row addressing for the plain sweeps; the extended ones measured 4-5% slower
  // with it (256^3 with sources: 2551 vs 2420 us)
  constexpr bool kRows = EXT == 0 && WALLS != 2;
  const int nbx = gridDim.x;
  const int tile = blockIdx.x + nbx * blockIdx.y;
  const int bx = tile % nbx, by = tile / nbx;
  const int x = bx * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  const int r_end = min(by * rows + rows, ny * nz);
  for (int r = by * rows; r < r_end; ++r) {
    const int y = r % ny, z = r / ny;
    S hf[27], hg[27];
    node_pops<S, WALLS, PULL, kRows>(A, nb, plane, nx, ny, nz, pitch, x, y, z, hf, hg);
    Moments3 m;
    moments3<EXT>(hf, hg, prm, m, prm.Fx, prm.Fy, prm.Fz, prm.Q);
    const int64_t off = ((int64_t)z * ny + y) * pitch + x;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      fld[a * plane + off] = (S)(m.rho * m.u[a] * (m.u[a] * m.u[a] + 3.0 * (m.theta - 1.0 / 3.0)));
    if (EXT && prm.full) {
      const double T = EXT == 2 ? (m.e + prm.va * m.rho) / prm.cv : m.theta * prm.inv_R;
      fld[3 * plane + off] = (S)T;
#pragma unroll
      for (int a = 0; a < 3; ++a) fld[(4 + a) * plane + off] = (S)m.u[a];
      if (EXT == 2) fld[7 * plane + off] = (S)(m.e + m.theta);
    }
  }
}

// Two waves per SIMD fit the plain collision (223 VGPRs); the extended ones need more than 256
// registers and run one wave without spills (at two they spilled 228-252 bytes per lane and
// took 3368 / 4153 / 4434 us per 256^3 step with sources / transport control / van der Waals,
// against 2626 / 2909 / 3009 us at one wave).
template <typename S, int HALO, int WALLS, bool PULL, bool DIAG, int EXT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(EXT == 0 ? 2 : 1)))
k_ddf3_collide(const S* __restrict__ A, const S* __restrict__ nb, S* __restrict__ B, int nx,
               int ny, int nz, int64_t pitch, int64_t plane, DdfParams prm,
               const S* __restrict__ fld, int rows, double* __restrict__ partials) {
  constexpr bool kLean = EXT == 0 && WALLS != 2;  // see RestShift
  constexpr bool kRows = kLean;                   // scalar-base row addressing, as in the flux sweep
  __shared__ RestShift rs;
  if (kLean) rs.fill(prm);
  const int nbx = gridDim.x;
  const int tile = blockIdx.x + nbx * blockIdx.y;
  const int bx = tile % nbx, by = tile / nbx;
  const int x = bx * blockDim.x + threadIdx.x;
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (x < nx) {
    const int r_end = min(by * rows + rows, ny * nz);
    for (int r = by * rows; r < r_end; ++r) {
      const int y = r % ny, z = r / ny;
      S hf[27], hg[27];
      node_pops<S, WALLS, PULL, kRows>(A, nb, plane, nx, ny, nz, pitch, x, y, z, hf, hg);
      Moments3 m;
      moments3<EXT>(hf, hg, prm, m, prm.Fx, prm.Fy, prm.Fz, prm.Q);
      const int64_t off = ((int64_t)z * ny + y) * pitch + x;
      // offset of the node k steps along axis a: periodic in x and z; in y periodic, or the
      // nearest fluid row beyond a wall (zero-order ghosts, Sec. III A)
      // (|k| <= 2: two conditional wraps cover lattices down to one node along the axis)
      auto wrap = [](int v, int n) {
        if (v < 0) v += n;
        if (v < 0) v += n;
        if (v >= n) v -= n;
        if (v >= n) v -= n;
        return v;
      };
      auto at = [&](int a, int k) -> int64_t {
        int xx = x, yy = y, zz = z;
        if (a == 0) xx = wrap(x + k, nx);
        if (a == 1) {
          yy = y + k;
          if (WALLS)
            yy = yy < 0 ? 0 : (yy > ny - 1 ? ny - 1 : yy);
          else
            yy = wrap(yy, ny);
        }
        if (a == 2) zz = wrap(z + k, nz);
        return ((int64_t)zz * ny + yy) * pitch + xx;
      };
      double ph[3] = {0.0, 0.0, 0.0};
      if (prm.phi) {
        const double inv_rho = 1.0 / m.rho;
        if constexpr (HALO == 1) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const S* F = fld + a * plane;
            const double d = 0.5 * ((double)F[at(a, 1)] - (double)F[at(a, -1)]);
            ph[a] = -d * inv_rho;
          }
        } else {
          // the five field values of each axis, all loaded before the side is chosen: the
          // empty asm uses them, so the compiler cannot move each load into the one branch of
          // the choice that needs it (and wait for it there)
          S v[3][5];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            const S* F = fld + a * plane;
            v[a][0] = F[at(a, -2)];
            v[a][1] = F[at(a, -1)];
            v[a][2] = F[off];
            v[a][3] = F[at(a, 1)];
            v[a][4] = F[at(a, 2)];
          }
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            asm volatile("" ::"v"(v[a][0]), "v"(v[a][1]), "v"(v[a][2]), "v"(v[a][3]),
                         "v"(v[a][4]));
            // the upwind side follows u_a; on the boundary planes of NEQ walls the wall's
            // velocity (normal component zero: central in y there)
            double key = m.u[a];
            if (WALLS == 2 && (y == 0 || y == ny - 1)) key = prm.uw[y == 0 ? 0 : 1][a];
            const double d = upwind_or_central((double)v[a][0], (double)v[a][1], (double)v[a][2],
                                               (double)v[a][3], (double)v[a][4], key);
            ph[a] = -d * inv_rho;
          }
        }
      }
      double gT[3] = {0.0, 0.0, 0.0}, gh[3] = {0.0, 0.0, 0.0}, divu = 0.0;
      if (EXT && prm.full) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          gT[a] = 0.5 * ((double)fld[3 * plane + at(a, 1)] - (double)fld[3 * plane + at(a, -1)]);
          divu += 0.5 * ((double)fld[(4 + a) * plane + at(a, 1)] -
                         (double)fld[(4 + a) * plane + at(a, -1)]);
          if (EXT == 2)
            gh[a] = 0.5 * ((double)fld[7 * plane + at(a, 1)] - (double)fld[7 * plane + at(a, -1)]);
        }
      }
      const double* w2 = kLean ? rs.at_row() : prm.wf;
      if constexpr (kRows) {
        S* out = B + ((int64_t)z * ny + y) * pitch;  // row base (wave-uniform)
        const uint32_t xo = fresh((uint32_t)sizeof(S) * x);
        int64_t pl = plane;
        asm volatile("" : "+s"(pl));
        collide3<EXT>(hf, hg, m, ph, gT, gh, divu, prm, w2, kLean ? w2 + 27 : prm.wg,
                      [&](int k, double t) { gstore_nt(at_byte(sbase(out + k * pl), xo), (S)t); });
      } else {
        S* out = B + off;
        collide3<EXT>(hf, hg, m, ph, gT, gh, divu, prm, w2, prm.wg,
                      [&](int k, double t) { store_nt(out + k * plane, (S)t); });
      }
      if (DIAG) {
        acc[0] += m.rho;
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[1 + a] += m.rho * m.u[a];
        const double u2 = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
        acc[4] += m.rho * (m.e + 0.5 * u2);
      }
    }
  }
  if (DIAG) block_sum_store<kDiagValues>(acc, partials + (int64_t)tile * kDiagValues);
}

// ---- one-launch step --------------------------------------------------------------------------
// With the central derivative of Phi (any collision: sources, transport control, the van der
// Waals fluid, NEQ walls), the flux and collision sweeps are fused into one launch that marches
// along z. A workgroup owns a tile of kF3Cols columns by kF3Rows rows (one row per
// wavefront) and a range of planes. Per plane z
//   1. four wavefronts compute the fluxes of one halo piece each of plane z + 1: the rows below
//      and above the tile (wavefronts 1 and 2) or phi_x of the columns left and right of half of
//      its rows (wavefronts 0 and 3, one node per lane);
//   2. every wavefront pulls its own row of plane z + 1, computes the moments and fluxes;
//   3. swaps populations with LDS: reads those of plane z (pulled one plane earlier) and writes
//      those of plane z + 1 in their place;
//   4. collides its row of plane z and stores it;
// and one barrier per plane orders the flux buffers. Wavefronts w and w + 4 share a SIMD, so each
// SIMD carries one halo piece and two rows per plane and the collision arithmetic is spread
// evenly over the four SIMDs of a compute unit. Eight rows per tile amortise the two halo rows
// over eight (256^3 float32, eight against four rows: plain 1692 vs 1810 us, sources 1789 vs
// 2002, Pr 0.71 1863 vs 2103, van der Waals 1922 vs 2090, NEQ walls 1752 vs 1900); the float32
// populations of the eight rows take 108 KB of LDS, so one workgroup of eight wavefronts runs
// per compute unit (two per SIMD, as before with two workgroups of four). phi_x and phi_y go to
// two LDS buffers (planes z, z + 1), phi_z to a ring of three registers per column. float64
// populations are not held in LDS and are pulled again at step 3, from the caches. Fluxes and
// fields are rounded to the storage type as the two-sweep fields store them, so both paths give
// identical results. Traffic: the populations are read from memory once and written once per
// node (432 B in float32), against about 1.5x that for two sweeps.
constexpr int kF3Cols = 64;                // columns per tile (one wavefront row)
constexpr int kF3Rows = 8;                 // rows per tile = wavefronts per workgroup
constexpr int kF3Threads = kF3Rows * 64;   // one row per wavefront
constexpr int kF3Slots = 256;              // resident workgroups: 256 compute units x 1

// Workgroup sum of N doubles per thread over the kF3Rows wavefronts of a one-launch workgroup,
// in block_sum_store's order (wavefront sums, then the wavefronts in order); thread 0 writes
// out[0..N).
template <int N>
__device__ __forceinline__ void fused3_sum_store(double (&v)[N], double* out) {
  __shared__ double red[kF3Rows][N];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
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
      double t = 0.0;
      for (int w = 0; w < kF3Rows; ++w) t += red[w][k];
      out[k] = t;
    }
  }
}

// WALLS: 0 periodic in y, 1 bounce-back walls, 2 non-equilibrium extrapolation walls (boundary
// planes read from nb, rebuilt by k_ddf3_neq_rows, as in the two sweeps).
// EXT: 0 the plain collision, 1 the ideal gas with the uniform body force and heat source and,
// with TR, transport control (Prandtl number, bulk viscosity), 2 the van der Waals fluid (TR).
// TR: the transport terms, whose fields T, u_a (and for the van der Waals fluid the enthalpy h)
// are exchanged like the fluxes: x neighbours through LDS with the halo columns, y neighbours
// through LDS with the halo rows, z neighbours in a register ring. The shifted equilibria's
// second set of axis factors spills some 20 registers per lane (with TR about 30), and the step
// still beats the two sweeps (256^3 float32: sources about 2000 vs 2420 us, Pr 0.71 2110 vs
// 2645 us, van der Waals 2090 vs 2742 us).
// Fluxes and fields are kept in the storage type, as the two-sweep fields are.
template <typename S, int WALLS, bool PULL, bool DIAG, int EXT, bool TR>
__global__ void __launch_bounds__(kF3Threads) __attribute__((amdgpu_waves_per_eu(2)))
k_ddf3_fused(const S* __restrict__ A, const S* __restrict__ nb, S* __restrict__ B, int nx,
             int ny, int nz, int64_t pitch, int64_t plane, DdfParams prm, int nbx, int nby,
             int nzc, double* __restrict__ partials) {
  constexpr bool kLds = sizeof(S) == 4;  // populations kept in LDS between pull and collision
  constexpr int NR = kLds ? kF3Rows : 1, NQ = kLds ? 54 : 1;
  // fields: 0 T, 1 u along the exchange axis, 2 h (van der Waals)
  constexpr int NF = TR ? (EXT == 2 ? 3 : 2) : 1;
  constexpr int FR = TR ? kF3Rows : 1, FC = TR ? kF3Cols : 1;
  __shared__ RestShift rs;
  // flux buffers in float64 (0.5% faster for the plain step) unless the transport fields need the
  // LDS; either holds the fluxes rounded to the storage type
  using PT = std::conditional_t<TR, S, double>;
  __shared__ PT s_px[2][kF3Rows][kF3Cols + 2];  // phi_x of the tile rows, slot column + 1
  __shared__ PT s_py[2][kF3Rows + 2][kF3Cols];  // phi_y of rows y0 - 1 .. y0 + kF3Rows
  __shared__ S s_pop[NR][NQ][kF3Cols];          // each wavefront's row of one plane
  __shared__ S s_fx[2][NF][FR][FC + 2];         // T, u_x (, h) like phi_x
  __shared__ S s_fy[2][NF][FR + 2][FC];         // T, u_y (, h) like phi_y
  rs.fill(prm);
  const int T = nbx * nby;
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  const int tile = b % T, chunk = b / T;
  const int bx = tile % nbx, by = tile / nbx;
  const int zb = (int)((int64_t)chunk * nz / nzc);
  const int ze = (int)((int64_t)(chunk + 1) * nz / nzc);
  // wavefront index as a scalar: the rows and their addresses are then computed once per
  // wavefront instead of per lane
  const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int x0 = bx * kF3Cols, y0 = by * kF3Rows;
  const int ncols = min(kF3Cols, nx - x0);
  const bool col_ok = lane < ncols;
  const int x = col_ok ? x0 + lane : x0 + ncols - 1;  // idle lanes repeat the last column
  // own row; past the last row of the lattice (not collided) its periodic image, or the last
  // row inside the walls, whose phi_y the row below takes as its neighbour's
  const bool row_ok = y0 + wv < ny;
  const int y = row_ok ? y0 + wv : (WALLS ? ny - 1 : (y0 + wv) % ny);
  // halo piece. Wavefronts 1, 2: row y0 - 1 or y0 + kF3Rows (periodic, or the nearest row
  // inside the walls: zero-order ghosts, Sec. III A). Wavefronts 0, 3: rows y0 + hr0 ..
  // y0 + hr0 + kF3Rows / 2 - 1, lane 2k + s: row hr0 + k, s = 0 the column left of the tile, 1
  // the column right of it (periodic); lanes past kF3Rows - 1 repeat lane 0 and store nothing.
  // The other wavefronts have no halo piece.
  const bool hrow = wv == 1 || wv == 2;
  int yr = wv == 1 ? y0 - 1 : y0 + kF3Rows;
  if (WALLS)
    yr = yr < 0 ? 0 : (yr > ny - 1 ? ny - 1 : yr);
  else
    yr = ((yr % ny) + ny) % ny;
  const int pyslot = wv == 1 ? 0 : kF3Rows + 1;
  const bool xrow = wv == 0 || wv == 3;
  const int hr0 = wv == 0 ? 0 : kF3Rows / 2;
  const int hk = lane < kF3Rows ? lane >> 1 : 0, hs = lane < kF3Rows ? lane & 1 : 0;
  const bool hx_ok = xrow && lane < kF3Rows && y0 + hr0 + hk < ny;
  const int yx = hx_ok ? y0 + hr0 + hk : y0;
  const int xx = hs ? (x0 + ncols == nx ? 0 : x0 + ncols) : (x0 == 0 ? nx - 1 : x0 - 1);
  const int pxslot = hs ? ncols + 1 : 0;
  auto wrapz = [&](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };
  auto phi_of = [](const Moments3& m, int a) {
    return (PT)(S)(m.rho * m.u[a] * (m.u[a] * m.u[a] + 3.0 * (m.theta - 1.0 / 3.0)));
  };
  // field f of the node along axis a (0 T, 1 u_a, 2 h), in the storage type as the two-sweep
  // fields store it
  auto field = [&](const Moments3& m, int f, int a) -> S {
    if (f == 0) return (S)(EXT == 2 ? (m.e + prm.va * m.rho) / prm.cv : m.theta * prm.inv_R);
    if (f == 1) return (S)m.u[a];
    return (S)(m.e + m.theta);
  };
  // all 54 loads of a pull are issued before the sums start: without the scheduling barrier
  // the compiler moves each load next to its single use and waits for it there, one load in
  // flight at a time
  auto moments = [&](const S (&hf)[27], const S (&hg)[27], Moments3& m) {
    __builtin_amdgcn_sched_barrier(0);
    moments3<EXT>(hf, hg, prm, m, prm.Fx, prm.Fy, prm.Fz, prm.Q);
  };
  // step 1 for plane z into flux buffer k
  auto halo = [&](int z, int k) {
    S hf[27], hg[27];
    Moments3 m;
    if (hrow) {
      node_pops<S, WALLS, PULL, true>(A, nb, plane, nx, ny, nz, pitch, x, yr, wrapz(z), hf, hg);
      moments(hf, hg, m);
      if (col_ok) {
        s_py[k][pyslot][lane] = phi_of(m, 1);
        if constexpr (TR) {
#pragma unroll
          for (int f = 0; f < NF; ++f) s_fy[k][f][pyslot][lane] = field(m, f, 1);
        }
      }
    } else if (xrow) {
      node_pops<S, WALLS, PULL, false>(A, nb, plane, nx, ny, nz, pitch, xx, yx, wrapz(z), hf, hg);
      moments(hf, hg, m);
      if (hx_ok) {
        s_px[k][hr0 + hk][pxslot] = phi_of(m, 0);
        if constexpr (TR) {
#pragma unroll
          for (int f = 0; f < NF; ++f) s_fx[k][f][hr0 + hk][pxslot] = field(m, f, 0);
        }
      }
    }
  };
  // step 2 for plane z into flux buffer k: own row pulled into hf, hg; phi_z and the fields
  // along z into zv
  auto own = [&](int z, int k, S (&hf)[27], S (&hg)[27], Moments3& m, PT (&zv)[NF + 1]) {
    node_pops<S, WALLS, PULL, true>(A, nb, plane, nx, ny, nz, pitch, x, y, wrapz(z), hf, hg);
    moments(hf, hg, m);
    if (col_ok) {
      s_px[k][wv][lane + 1] = phi_of(m, 0);
      s_py[k][wv + 1][lane] = phi_of(m, 1);
      if constexpr (TR) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          s_fx[k][f][wv][lane + 1] = field(m, f, 0);
          s_fy[k][f][wv + 1][lane] = field(m, f, 1);
        }
      }
    }
    zv[0] = phi_of(m, 2);
    if constexpr (TR) {
#pragma unroll
      for (int f = 0; f < NF; ++f) zv[1 + f] = field(m, f, 2);
    }
  };
  auto put = [&](const S (&hf)[27], const S (&hg)[27]) {
    if constexpr (kLds) {
#pragma unroll
      for (int i = 0; i < 27; ++i) {
        s_pop[wv][i][lane] = hf[i];
        s_pop[wv][27 + i][lane] = hg[i];
      }
    }
  };
  double acc[kDiagValues] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (ze > zb) {
    Moments3 m0;
    PT zv_prv[NF + 1], zv_cur[NF + 1];  // phi_z and the fields of planes z - 1, z
    {
      S hf[27], hg[27];
      Moments3 m;
      own(zb - 1, 1, hf, hg, m, zv_prv);  // below the range (buffer 1 rewritten below)
      halo(zb, 0);
      own(zb, 0, hf, hg, m0, zv_cur);
      put(hf, hg);
    }
    __syncthreads();
    int kc = 0;  // flux buffer of plane z
    for (int z = zb; z < ze; ++z) {
      const int kn = kc ^ 1;
      halo(z + 1, kn);
      S hf[27], hg[27];
      PT zv_nxt[NF + 1];
      Moments3 m1;
      {
        S nf[27], ng[27];
        own(z + 1, kn, nf, ng, m1, zv_nxt);
        if constexpr (kLds) {
#pragma unroll
          for (int i = 0; i < 27; ++i) {
            hf[i] = s_pop[wv][i][lane];
            hg[i] = s_pop[wv][27 + i][lane];
          }
          put(nf, ng);
        } else {
          node_pops<S, WALLS, PULL, true>(A, nb, plane, nx, ny, nz, pitch, x, y, z, hf, hg);
        }
      }
      if (row_ok) {
        const double inv_rho = 1.0 / m0.rho;
        double ph[3];
        ph[0] = -(0.5 * ((double)s_px[kc][wv][lane + 2] - (double)s_px[kc][wv][lane])) * inv_rho;
        ph[1] = -(0.5 * ((double)s_py[kc][wv + 2][lane] - (double)s_py[kc][wv][lane])) * inv_rho;
        ph[2] = -(0.5 * ((double)zv_nxt[0] - (double)zv_prv[0])) * inv_rho;
        // derivatives of the fields, in the two sweeps' order: gT and gh per axis, div u summed
        // over x, y, z
        double gT[3] = {0.0, 0.0, 0.0}, gh[3] = {0.0, 0.0, 0.0}, divu = 0.0;
        if constexpr (TR) {
          auto dx = [&](int f) {
            return 0.5 * ((double)s_fx[kc][f][wv][lane + 2] - (double)s_fx[kc][f][wv][lane]);
          };
          auto dy = [&](int f) {
            return 0.5 * ((double)s_fy[kc][f][wv + 2][lane] - (double)s_fy[kc][f][wv][lane]);
          };
          auto dz = [&](int f) { return 0.5 * ((double)zv_nxt[1 + f] - (double)zv_prv[1 + f]); };
          gT[0] = dx(0);
          divu += dx(1);
          gT[1] = dy(0);
          divu += dy(1);
          gT[2] = dz(0);
          divu += dz(1);
          if constexpr (EXT == 2) {
            gh[0] = dx(2);
            gh[1] = dy(2);
            gh[2] = dz(2);
          }
        }
        const double* w2 = rs.at_row();
        S* out = B + ((int64_t)z * ny + y) * pitch;  // row base (wave-uniform)
        const uint32_t xo = fresh((uint32_t)sizeof(S) * x);
        int64_t pl = plane;
        asm volatile("" : "+s"(pl));
        collide3<EXT, TR>(hf, hg, m0, ph, gT, gh, divu, prm, w2, w2 + 27,
                          [&](int k, double t) {
          if (col_ok) gstore_nt(at_byte(sbase(out + k * pl), xo), (S)t);
        });
        if (DIAG && col_ok) {
          acc[0] += m0.rho;
#pragma unroll
          for (int a = 0; a < 3; ++a) acc[1 + a] += m0.rho * m0.u[a];
          const double u2 = m0.u[0] * m0.u[0] + m0.u[1] * m0.u[1] + m0.u[2] * m0.u[2];
          acc[4] += m0.rho * (m0.e + 0.5 * u2);
        }
      }
      m0 = m1;
#pragma unroll
      for (int f = 0; f <= NF; ++f) {
        zv_prv[f] = zv_cur[f];
        zv_cur[f] = zv_nxt[f];
      }
      kc = kn;
      __syncthreads();
    }
  }
  if (DIAG) fused3_sum_store<kDiagValues>(acc, partials + (int64_t)blockIdx.x * kDiagValues);
}

// f <- f^eq, g <- g^eq of the initial fields (Fig. 1), shifted by the rest state.
template <typename S>
__global__ void k_init_ddf3(const double* __restrict__ rho, const double* __restrict__ u,
                            const double* __restrict__ T, S* __restrict__ A, int nx, int64_t nodes,
                            int64_t pitch, int64_t plane, DdfParams prm) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  double theta = prm.R * T[n], e = prm.cv * T[n];
  if (prm.eos) {  // van der Waals: theta = P / rho, e = c_v T - a rho
    theta = prm.R * T[n] / (1.0 - prm.vb * rho[n]) - prm.va * rho[n];
    e -= prm.va * rho[n];
  }
  const double uu[3] = {u[n], u[nodes + n], u[2 * nodes + n]};
  Axis X[3];
  for (int a = 0; a < 3; ++a) axis_eq(uu[a], theta, X[a]);
  for (int i = 0; i < 27; ++i) {
    double fe, ge;
    equilibria3(rho[n], e, i, X, fe, ge);
    A[i * plane + off] = (S)(fe - prm.wf[i]);
    A[(27 + i) * plane + off] = (S)(ge - prm.wg[i]);
  }
}

// rho, u, T and rho E of the stored post-collision state: the closure with the sources of the
// collision that produced it negated (prm.Fx, prm.Fy, prm.Fz, prm.Q hold them).
template <typename S>
__global__ void k_moments_ddf3(const S* __restrict__ A, int nx, int64_t nodes, int64_t pitch,
                               int64_t plane, DdfParams prm, double* __restrict__ rho,
                               double* __restrict__ u, double* __restrict__ T,
                               double* __restrict__ edens) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nodes) return;
  const int64_t off = (n / nx) * pitch + (n % nx);
  S hf[27], hg[27];
  for (int i = 0; i < 27; ++i) {
    hf[i] = A[i * plane + off];
    hg[i] = A[(27 + i) * plane + off];
  }
  Moments3 m;
  if (prm.eos) moments3<2>(hf, hg, prm, m, -prm.Fx, -prm.Fy, -prm.Fz, -prm.Q);
  else moments3<1>(hf, hg, prm, m, -prm.Fx, -prm.Fy, -prm.Fz, -prm.Q);
  rho[n] = m.rho;
  for (int a = 0; a < 3; ++a) u[a * nodes + n] = m.u[a];
  T[n] = prm.eos ? (m.e + prm.va * m.rho) / prm.cv : m.theta / prm.R;
  edens[n] = m.rho * (m.e + 0.5 * (m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2]));
}

__global__ void k_ddf3_rest_state(DdfParams prm, double* __restrict__ out) {
  Axis X[3];
  for (int a = 0; a < 3; ++a) axis_eq(0.0, prm.R, X[a]);
  for (int i = 0; i < 27; ++i) equilibria3(1.0, prm.cv, i, X, out[i], out[27 + i]);
}

// ---- launchers ------------------------------------------------------------------------------
static inline unsigned nblk3(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

hipError_t launch_ddf3_rest_state(const DdfParams& prm, double* out, hipStream_t s) {
  k_ddf3_rest_state<<<1, 1, 0, s>>>(prm, out);
  return hipGetLastError();
}

hipError_t launch_init_ddf3(int kind, const double* rho, const double* u, const double* T,
                            void* A, const Layout& L, const DdfParams& prm, hipStream_t s) {
  if (kind == 0)
    k_init_ddf3<float><<<nblk3(L.nodes()), kBlock, 0, s>>>(rho, u, T, static_cast<float*>(A), L.nx, L.nodes(), L.pitch, L.plane, prm);
  else
    k_init_ddf3<double><<<nblk3(L.nodes()), kBlock, 0, s>>>(rho, u, T, static_cast<double*>(A), L.nx, L.nodes(), L.pitch, L.plane, prm);
  return hipGetLastError();
}

hipError_t launch_moments_ddf3(int kind, const void* A, const Layout& L, const DdfParams& prm,
                               double* rho, double* u, double* T, double* edens, hipStream_t s) {
  if (kind == 0)
    k_moments_ddf3<float><<<nblk3(L.nodes()), kBlock, 0, s>>>(static_cast<const float*>(A), L.nx, L.nodes(), L.pitch, L.plane, prm, rho, u, T, edens);
  else
    k_moments_ddf3<double><<<nblk3(L.nodes()), kBlock, 0, s>>>(static_cast<const double*>(A), L.nx, L.nodes(), L.pitch, L.plane, prm, rho, u, T, edens);
  return hipGetLastError();
}

// The isothermal grid (one row per workgroup at 256^3), with at least two rows per workgroup:
// at 256^3 float32, 1 row -> 2256-2269 us per step, 2 -> 2222-2225, 4 -> 2223; 128-wide
// workgroups 2266-2297, 64-wide 2437-2472.
Grid make_grid_ddf3(const Layout& L) {
  Grid G = make_grid(L);
  if (G.rows < 2) G.rows = 2;
#ifdef LBM_TUNING_ENV
  if (const char* v = getenv("LBM_DDF3_ROWS")) G.rows = atoi(v);
#endif
  fit_rows(G, (int64_t)L.ny * L.nz);
  return G;
}

template <typename Fn>
static void flag(bool b, Fn&& fn) {
  if (b)
    fn(std::true_type{});
  else
    fn(std::false_type{});
}

// The collision variant as a template argument: 0 plain, 1 sources / transport control (ideal
// gas), 2 van der Waals fluid.
template <typename Fn>
static void ext_kind(const DdfParams& prm, Fn&& fn) {
  if (prm.eos)
    fn(std::integral_constant<int, 2>{});
  else if (prm.ext())
    fn(std::integral_constant<int, 1>{});
  else
    fn(std::integral_constant<int, 0>{});
}

// Non-equilibrium extrapolation walls (App. B; the D2Q9 form is k_ddf_neq_rows): the
// pre-collision populations of the boundary planes B (y = 0 and ny - 1, on the walls) are
// f^eq(rho_B, u_W, T_W) + f_N - f^eq(rho_N, u_N, T_N), N the neighbouring plane (1, ny - 2)
// pulled like any fluid node, rho_B the pressure-continued or the literal density
// (neq_wall_state); EXT = 2: the van der Waals closure at N and at the wall. One thread per
// (x, z, side); written to nb as node_pops reads it.
template <typename S, bool PULL, int EXT>
__global__ void __launch_bounds__(kBlock)
k_ddf3_neq_rows(const S* __restrict__ A, int nx, int ny, int nz, int64_t pitch, int64_t plane,
                DdfParams prm, S* __restrict__ nb) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= 2 * (int64_t)nz * nx) return;
  const int x = (int)(n % nx);
  const int64_t t = n / nx;
  const int z = (int)(t % nz), side = (int)(t / nz);
  const int N = side ? ny - 2 : 1;
  S hf[27], hg[27];
  gather27<S, true, PULL, false>(A, plane, nx, ny, nz, pitch, x, N, z, hf, hg);
  Moments3 m;
  moments3<EXT == 2 ? 2 : 0>(hf, hg, prm, m, 0.0, 0.0, 0.0, 0.0);
  constexpr bool VDW = EXT == 2;
  const double TN = node_temperature<VDW>(prm, m.rho, m.e, m.theta);
  double rhoB, thetaW, eW;
  neq_wall_state<VDW>(prm, side, m.rho, TN, m.rho * m.theta, rhoB, thetaW, eW);
  const double uW[3] = {prm.uw[side][0], prm.uw[side][1], prm.uw[side][2]};
  Axis X[3], XB[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    axis_eq(m.u[a], m.theta, X[a]);
    axis_eq(uW[a], thetaW, XB[a]);
  }
  const int64_t nbp = (int64_t)nz * pitch;
  const int64_t o = (int64_t)side * 54 * nbp + (int64_t)z * pitch + x;
  for (int i = 0; i < 27; ++i) {
    double feN, geN, feB, geB;
    equilibria3(m.rho, m.e, i, X, feN, geN);
    equilibria3(rhoB, eW, i, XB, feB, geB);
    const double f = (double)hf[i] + prm.wf[i], g = (double)hg[i] + prm.wg[i];
    nb[o + i * nbp] = (S)(feB + (f - feN) - prm.wf[i]);
    nb[o + (27 + i) * nbp] = (S)(geB + (g - geN) - prm.wg[i]);
  }
}

// The wall type as a template argument: 0 periodic in y, 1 bounce-back, 2 NEQ extrapolation.
template <typename Fn>
static void wall_kind(bool walls, const DdfParams& prm, Fn&& fn) {
  if (!walls)
    fn(std::integral_constant<int, 0>{});
  else if (prm.neq)
    fn(std::integral_constant<int, 2>{});
  else
    fn(std::integral_constant<int, 1>{});
}

// Shape of the one-launch step: tiles of kF3Cols x kF3Rows nodes, each with its planes split
// into nzc balanced ranges. nzc minimises the launch's rounds of kF3Slots resident workgroups
// times the planes per range (plus the two flux planes a range starts with).
struct Fused3 {
  int nbx, nby, nzc;
  int64_t blocks() const { return (int64_t)nbx * nby * nzc; }
};

static Fused3 fused3_shape(const Layout& L) {
  Fused3 F;
  F.nbx = (L.nx + kF3Cols - 1) / kF3Cols;
  F.nby = (L.ny + kF3Rows - 1) / kF3Rows;
  F.nzc = 1;
  const int64_t T = (int64_t)F.nbx * F.nby;
  int64_t best = -1;
  for (int c = 1; c <= std::min(L.nz, 64); ++c) {
    if (T * c > (int64_t)1 << 30) break;
    const int64_t cost = ((T * c + kF3Slots - 1) / kF3Slots) * ((L.nz + c - 1) / c + 2);
    if (best < 0 || cost < best) {
      best = cost;
      F.nzc = c;
    }
  }
  return F;
}

// The upwind collision sweep takes one row per workgroup (256^3 float32 with upwind Phi: 1 row
// 2080 us, 2 rows 2151, 4 rows 2170; the transport-control and van der Waals sweeps are even
// between 2 and 4 rows and keep the plan's).
static Grid upwind3_grid(const Layout& L, const Grid& G) {
  Grid U = G;
  U.rows = 1;
  fit_rows(U, (int64_t)L.ny * L.nz);
  return U;
}

int64_t ddf3_max_records(const Layout& L, const Grid& G) {
  return std::max<int64_t>(fused3_shape(L).blocks(), upwind3_grid(L, G).blocks());
}

static bool fused3_ok(const DdfParams& prm) { return prm.phi == 1; }

template <typename S>
static void ddf3_step(bool walls, bool pull, const S* A, S* B, const Layout& L, const Grid& G0,
                      const DdfParams& prm, double* fld64, S* nb, double* partials,
                      int* records, hipStream_t s) {
  if (walls && prm.neq) {
    const unsigned nblk = (unsigned)((2 * (int64_t)L.nz * L.nx + kBlock - 1) / kBlock);
    flag(pull, [&](auto Pl) {
      flag(prm.eos != 0, [&](auto V) {
        k_ddf3_neq_rows<S, decltype(Pl)::value, decltype(V)::value ? 2 : 0>
            <<<nblk, kBlock, 0, s>>>(A, L.nx, L.ny, L.nz, L.pitch, L.plane, prm, nb);
      });
    });
  }
  if (fused3_ok(prm)) {
    const Fused3 F = fused3_shape(L);
    *records = (int)F.blocks();
    wall_kind(walls, prm, [&](auto W) {
      flag(pull, [&](auto Pl) {
        flag(partials != nullptr, [&](auto Dg) {
          constexpr int w = decltype(W)::value;
          constexpr bool pl = decltype(Pl)::value, dg = decltype(Dg)::value;
          const unsigned nb_blocks = (unsigned)F.blocks();
          auto go = [&](auto kern) {
            kern<<<nb_blocks, kF3Threads, 0, s>>>(A, nb, B, L.nx, L.ny, L.nz, L.pitch, L.plane, prm,
                                              F.nbx, F.nby, F.nzc, partials);
          };
          if (prm.eos)
            go(k_ddf3_fused<S, w, pl, dg, 2, true>);
          else if (prm.full)
            go(k_ddf3_fused<S, w, pl, dg, 1, true>);
          else if (prm.src)
            go(k_ddf3_fused<S, w, pl, dg, 1, false>);
          else
            go(k_ddf3_fused<S, w, pl, dg, 0, false>);
        });
      });
    });
    return;
  }
  const Grid Gs = prm.phi == 2 ? upwind3_grid(L, G0) : G0;
  *records = Gs.blocks();
  dim3 grid(Gs.nbx, Gs.nby), block(Gs.bx);
  S* fld = reinterpret_cast<S*>(fld64);  // 8 planes of the storage type
  wall_kind(walls, prm, [&](auto W) {
    flag(pull, [&](auto Pl) {
      ext_kind(prm, [&](auto E) {
        constexpr int w = decltype(W)::value, e = decltype(E)::value;
        constexpr bool pl = decltype(Pl)::value;
        {
          // the fields are read only for Phi and for transport control
          if (prm.phi || (e && prm.full))
            k_ddf3_flux<S, w, pl, e><<<grid, block, 0, s>>>(A, nb, L.nx, L.ny, L.nz, L.pitch,
                                                            L.plane, prm, Gs.rows, fld);
          flag(partials != nullptr, [&](auto Dg) {
            constexpr bool dg = decltype(Dg)::value;
            if (prm.phi == 2)
              k_ddf3_collide<S, 2, w, pl, dg, e><<<grid, block, 0, s>>>(
                  A, nb, B, L.nx, L.ny, L.nz, L.pitch, L.plane, prm, fld, Gs.rows, partials);
            else
              k_ddf3_collide<S, 1, w, pl, dg, e><<<grid, block, 0, s>>>(
                  A, nb, B, L.nx, L.ny, L.nz, L.pitch, L.plane, prm, fld, Gs.rows, partials);
          });
        }
      });
    });
  });
}

hipError_t launch_ddf3(int kind, bool walls, bool pull, const void* A, void* B, const Layout& L,
                       const Grid& G, const DdfParams& prm, double* fld, void* nb,
                       double* partials, int* records, hipStream_t s) {
  if (prm.neq && (!walls || !nb || L.ny < 3 || prm.src))
    return hipErrorInvalidValue;
  int rec = 0;
  if (kind == 0)
    ddf3_step<float>(walls, pull, static_cast<const float*>(A), static_cast<float*>(B), L, G,
                     prm, fld, static_cast<float*>(nb), partials, &rec, s);
  else
    ddf3_step<double>(walls, pull, static_cast<const double*>(A), static_cast<double*>(B), L, G,
                      prm, fld, static_cast<double*>(nb), partials, &rec, s);
  if (records) *records = rec;
  return hipGetLastError();
}

}  // namespace lbm
