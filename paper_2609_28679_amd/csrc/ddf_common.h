// Device helpers of the double-distribution (ideal gas) kernels, D2Q9.
#pragma once

#include "device_common.h"

namespace lbm {

// Per-axis factors of the product-form equilibria at velocity component v and reference
// temperature theta (Sec. II C), indexed by k = c + 1:
//   psi_c = Psi(c; v, theta + v^2):  1 - theta - v^2 (c = 0), (theta + v^2 +- v)/2 (c = +-1)
//   chi_c = Psi(c; O, O^2) applied to v^2/2 with O = theta d/dv + v:
//           a0 - a2 (c = 0), (a2 +- a1)/2 (c = +-1), where a0 = v^2/2, a1 = O a0 = theta v + v^3/2,
//           a2 = O^2 a0 = theta^2 + 5/2 theta v^2 + v^4/2.
// Then f_i^eq = rho psi_x psi_y and, the operators acting on E = e + u_x^2/2 + u_y^2/2,
// g_i^eq = rho (e psi_x psi_y + chi_x psi_y + psi_x chi_y).
struct Axis {
  double psi[3];
  double chi[3];
};

__device__ __forceinline__ void axis_eq(double v, double theta, Axis& a) {
  const double v2 = v * v;
  a.psi[1] = 1.0 - theta - v2;
  a.psi[2] = 0.5 * (theta + v2 + v);
  a.psi[0] = 0.5 * (theta + v2 - v);
  const double a0 = 0.5 * v2;
  const double a1 = theta * v + 0.5 * v2 * v;
  const double a2 = theta * theta + 2.5 * theta * v2 + 0.5 * v2 * v2;
  a.chi[1] = a0 - a2;
  a.chi[2] = 0.5 * (a2 + a1);
  a.chi[0] = 0.5 * (a2 - a1);
}

__device__ __forceinline__ void equilibria(double rho, double ux, double uy, double theta,
                                           double e, double (&fe)[9], double (&ge)[9]) {
  Axis X, Y;
  axis_eq(ux, theta, X);
  axis_eq(uy, theta, Y);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int a = i % 3, b = i / 3;
    const double pp = X.psi[a] * Y.psi[b];
    fe[i] = rho * pp;
    ge[i] = rho * (e * pp + X.chi[a] * Y.psi[b] + X.psi[a] * Y.chi[b]);
  }
}

struct Moments {
  double rho, ux, uy, theta, e;
};

// rho = sum f, rho u = sum c f, rho E = sum g; T = (E - u^2/2)/c_v and theta = P/rho = R T.
// VDW: van der Waals closure (Eq. lbm_temp); the ideal-gas instantiations carry none of it.
// With sources (SRC) the half-step terms of Sec. II C enter: rho u = sum c f + sF/2 and
// rho E = sum g + (u.sF + sQ)/2, (sF, sQ) = (F, Q) of the collision that follows. The
// post-collision state (whose sums carry a whole step of the sources) gives the same moments
// with (sF, sQ) = -(F, Q) of the collision that produced it.
template <bool SRC = false, bool VDW = false>
__device__ __forceinline__ void moments_closure(const double (&f)[9], const double (&g)[9],
                                                const DdfParams& p, Moments& m, double sFx = 0.0,
                                                double sFy = 0.0, double sQ = 0.0) {
  const double rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  double jx = (f[2] + f[5] + f[8]) - (f[0] + f[3] + f[6]);
  double jy = (f[6] + f[7] + f[8]) - (f[0] + f[1] + f[2]);
  double rE = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  if (SRC) {
    jx += 0.5 * sFx;
    jy += 0.5 * sFy;
  }
  const double inv = 1.0 / rho;
  m.rho = rho;
  m.ux = jx * inv;
  m.uy = jy * inv;
  if (SRC) rE += 0.5 * ((m.ux * sFx + m.uy * sFy) + sQ);
  m.e = rE * inv - 0.5 * (m.ux * m.ux + m.uy * m.uy);  // specific internal energy
  if (VDW) {  // van der Waals: T = (e + a rho) / c_v (Eq. lbm_temp), theta = P / rho
    const double T = (m.e + p.va * rho) / p.cv;
    m.theta = p.R * T / (1.0 - p.vb * rho) - p.va * rho;
  } else {
    m.theta = p.r_cv * m.e;  // ideal gas: theta = R T = (R / c_v) e
  }
}

// The same closure from the stored deviations h = f - w, g - v of the shifted storage: the
// sums run over the deviations and add the rest totals sum w, sum v once (p.wsum_f, p.wsum_g);
// the momentum sums need no shift, w being even in each velocity component.
template <bool SRC = false, bool VDW = false, typename R>
__device__ __forceinline__ void moments_closure_dev(const R (&hf)[9], const R (&hg)[9],
                                                    const DdfParams& p, Moments& m,
                                                    double sFx = 0.0, double sFy = 0.0,
                                                    double sQ = 0.0) {
  double f[9], g[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    f[i] = (double)hf[i];
    g[i] = (double)hg[i];
  }
  const double rho =
      (((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8]) + p.wsum_f;
  double jx = (f[2] + f[5] + f[8]) - (f[0] + f[3] + f[6]);
  double jy = (f[6] + f[7] + f[8]) - (f[0] + f[1] + f[2]);
  double rE =
      (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8]) + p.wsum_g;
  if (SRC) {
    jx += 0.5 * sFx;
    jy += 0.5 * sFy;
  }
  const double inv = 1.0 / rho;
  m.rho = rho;
  m.ux = jx * inv;
  m.uy = jy * inv;
  if (SRC) rE += 0.5 * ((m.ux * sFx + m.uy * sFy) + sQ);
  m.e = rE * inv - 0.5 * (m.ux * m.ux + m.uy * m.uy);
  if (VDW) {
    const double T = (m.e + p.va * rho) / p.cv;
    m.theta = p.R * T / (1.0 - p.vb * rho) - p.va * rho;
  } else {
    m.theta = p.r_cv * m.e;
  }
}

// Temperature of a node from its moments (ideal gas: theta / R; van der Waals: Eq. lbm_temp).
template <bool VDW>
__device__ __forceinline__ double node_temperature(const DdfParams& p, double rho, double e,
                                                   double theta) {
  return VDW ? (e + p.va * rho) / p.cv : theta * p.inv_R;
}

// State of a boundary node of the non-equilibrium extrapolation walls (App. B) next to the
// fluid node N (density rhoN, temperature TN, pressure PN): the density rho_B and the wall
// equilibrium's theta_W = P(rho_B, T_W)/rho_B and e_W = e(rho_B, T_W) at the wall temperature
// of `side`. rho_B = rho_N with p.neq_literal, otherwise the density that continues P_N to the
// wall: rho_N T_N / T_W for the ideal gas; for the van der Waals fluid (VDW) the root of
// P(rho, T_W) = P_N on a supercritical isotherm (T_W > T_cr, checked at context creation),
// where P is strictly increasing on 0 < rho < 1/b: Newton steps from rho_N kept inside a
// bisection bracket, until the iterate repeats or 100 steps.
template <bool VDW>
__device__ __forceinline__ void neq_wall_state(const DdfParams& p, int side, double rhoN,
                                               double TN, double PN, double& rhoB,
                                               double& thetaW, double& eW) {
  const double TW = p.Tw[side];
  if constexpr (VDW) {
    rhoB = rhoN;
    if (!p.neq_literal) {
      const double RT = p.R * TW;
      double lo = 0.0, hi = 1.0 / p.vb, r = rhoN;
      if (!(r > lo && r < hi)) r = 0.5 * hi;
      for (int it = 0; it < 100; ++it) {
        const double omb = 1.0 - p.vb * r;
        const double P = r * RT / omb - p.va * r * r;
        if (P > PN) hi = r;
        else lo = r;
        double rn = r - (P - PN) / (RT / (omb * omb) - 2.0 * p.va * r);
        if (!(rn > lo && rn < hi)) rn = 0.5 * (lo + hi);
        if (rn == r) break;
        r = rn;
      }
      rhoB = r;
    }
    thetaW = p.R * TW / (1.0 - p.vb * rhoB) - p.va * rhoB;
    eW = p.cv * TW - p.va * rhoB;
  } else {
    (void)PN;
    rhoB = p.neq_literal ? rhoN : rhoN * TN / TW;
    thetaW = p.R * TW;
    eW = p.cv * TW;
  }
}

// Pull of the nine populations of one distribution at node (x, row): f_i = A_i(x - c_i).
// top/bot: the row touches the upper/lower half-way bounce-back wall.
template <typename S>
__device__ __forceinline__ void gather9(const S* __restrict__ A, int64_t plane, int64_t r0,
                                        int64_t rm, int64_t rp, int x, int xm, int xp,
                                        bool top, bool bot, S (&h)[9]) {
  h[3] = A[3 * plane + r0 + xp];
  h[4] = A[4 * plane + r0 + x];
  h[5] = A[5 * plane + r0 + xm];
  if (top) {
    h[0] = A[8 * plane + r0 + x];
    h[1] = A[7 * plane + r0 + x];
    h[2] = A[6 * plane + r0 + x];
  } else {
    h[0] = A[0 * plane + rp + xp];
    h[1] = A[1 * plane + rp + x];
    h[2] = A[2 * plane + rp + xm];
  }
  if (bot) {
    h[6] = A[2 * plane + r0 + x];
    h[7] = A[1 * plane + r0 + x];
    h[8] = A[0 * plane + r0 + x];
  } else {
    h[6] = A[6 * plane + rm + xp];
    h[7] = A[7 * plane + rm + x];
    h[8] = A[8 * plane + rm + xm];
  }
}

// Second-order one-sided difference on the upwind side of u (central when u = 0). All three
// stencils are formed and one is selected: written as branches, the compiler moved each field
// load into the branch that uses it and waited for it there.
__device__ __forceinline__ double upwind_or_central(double pm2, double pm1, double p0, double pp1,
                                                    double pp2, double u) {
  const double up = 0.5 * (3.0 * p0 - 4.0 * pm1 + pm2);
  const double un = -0.5 * (3.0 * p0 - 4.0 * pp1 + pp2);
  const double c = 0.5 * (pp1 - pm1);
  return u > 0.0 ? up : (u < 0.0 ? un : c);
}

// Collision of one node from its pre-collision populations held shifted by the rest state
// (hf = f - w, hg = g - v) and its moments m = {rho, u_x, u_y, theta, e, -, dT/dx, du_x/dx,
// dh/dx} (the derivatives on the extended path only);
// Phi_xx, Phi_yy include dt = 1. For every i the sink receives the post-collision values and
// the equilibria, all shifted: sink(i, f~ - w, f^eq - w, g~ - v, g^eq - v).
// Without the extended path (EXT = false) f* = rho prod Psi(u, theta + u^2 + Phi) and
// g* = g^eq. With it (Sec. II C) f* and g* are taken at the shifted state u* = u + F/rho,
// theta* = theta + alpha theta div u + (gamma - 1) Q/rho with gamma - 1 = R/c_v (ideal gas),
// c_v T* = e + Q/rho - F.F/(2 rho^2), and g* gains c_i.q^c/2 on the four velocities with
// |c_i| = 1, q^c = P (c_p - k/mu) grad T (the ideal-gas form of P (grad h - (k/mu) grad T));
// m[6], m[7], dTdy, duydy are used only when p.full; for the van der Waals fluid (VDW)
// gamma - 1 and alpha are per node and q^c = P (grad h - (k/mu) grad T) with h = e + P/rho
// (m[8], dhdy).
template <bool EXT = false, bool VDW = false, typename R, typename Sink>
__device__ __forceinline__ void collide_ddf(const R (&hf)[9], const R (&hg)[9],
                                            const double* m, double phxx, double phyy,
                                            double dTdy, double duydy, double dhdy,
                                            const DdfParams& p, Sink&& sink) {
  const double rho = m[0], theta = m[3], e = m[4];
  const double P = rho * theta;
  Axis X, Y;
  axis_eq(m[1], theta, X);
  axis_eq(m[2], theta, Y);
  // shifted state: the factors of f*, g* (the unshifted ones without the extended path)
  Axis XS = X, YS = Y;
  double es = e, qx = 0.0, qy = 0.0;
  if (EXT) {
    const double inv = 1.0 / rho;
    double thetas;
    if constexpr (VDW) {  // van der Waals: gamma - 1 = R / ((1 - b rho) c_v), alpha and q^c per node
      const double omb = 1.0 - p.vb * rho;
      const double T = (e + p.va * rho) / p.cv;
      const double cs2 = p.R * T / (omb * omb) - 2.0 * p.va * rho +
                         T * p.R * p.R / (p.cv * omb * omb);
      const double alpha = 2.0 - rho * cs2 / P - p.eta;  // (D+2)/D - rho c_s^2 / P - eta/mu
      thetas = theta + p.R / (omb * p.cv) * p.Q * inv + alpha * theta * (m[7] + duydy);
      qx = P * (m[8] - p.kmu * m[6]);
      qy = P * (dhdy - p.kmu * dTdy);
    } else {
      thetas = theta + p.r_cv * p.Q * inv;
      if (p.full) {
        thetas += p.alpha * theta * (m[7] + duydy);
        qx = P * p.qc * m[6];
        qy = P * p.qc * dTdy;
      }
    }
    axis_eq(m[1] + p.Fx * inv, thetas, XS);
    axis_eq(m[2] + p.Fy * inv, thetas, YS);
    es = e + p.Q * inv - 0.5 * (p.Fx * p.Fx + p.Fy * p.Fy) * inv * inv;
  }
  // Psi(c; u*, theta* + u*^2 + Phi): psi* + Phi * (1/2, -1, 1/2)
  double sx[3], sy[3];
  sx[0] = XS.psi[0] + 0.5 * phxx;
  sx[1] = XS.psi[1] - phxx;
  sx[2] = XS.psi[2] + 0.5 * phxx;
  sy[0] = YS.psi[0] + 0.5 * phyy;
  sy[1] = YS.psi[1] - phyy;
  sy[2] = YS.psi[2] + 0.5 * phyy;
  const double omega = 2.0 * P / (2.0 * p.mu + P);  // 2 beta, beta = 1/(2 tau + 1), tau = mu/P
  const double keep = 1.0 - 0.5 * omega;            // 1 - beta
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int a = i % 3, b = i / 3;
    const double pp = X.psi[a] * Y.psi[b];
    const double hfe = rho * pp - p.wf[i];  // f^eq - w
    const double f = (double)hf[i];
    const double g = (double)hg[i];
    if (EXT) {
      const double fe = rho * pp;
      const double ge = rho * (e * pp + X.chi[a] * Y.psi[b] + X.psi[a] * Y.chi[b]);
      double gs = rho * (es * (XS.psi[a] * YS.psi[b]) + XS.chi[a] * YS.psi[b] +
                         XS.psi[a] * YS.chi[b]);
      if (i == 1) gs -= 0.5 * qy;  // c = (0, -1)
      if (i == 3) gs -= 0.5 * qx;  // c = (-1, 0)
      if (i == 5) gs += 0.5 * qx;  // c = (+1, 0)
      if (i == 7) gs += 0.5 * qy;  // c = (0, +1)
      const double hge = ge - p.wg[i];
      sink(i, f + omega * (hfe - f) + keep * (rho * (sx[a] * sy[b]) - fe), hfe,
           g + omega * (hge - g) + keep * (gs - ge), hge);
    } else {
      const double hge = rho * (e * pp + X.chi[a] * Y.psi[b] + X.psi[a] * Y.chi[b]) - p.wg[i];
      const double dstar = rho * (sx[a] * sy[b] - pp);  // f* - f^eq
      sink(i, f + omega * (hfe - f) + keep * dstar, hfe, g + omega * (hge - g), hge);
    }
  }
}

// Per-axis factors for one velocity component c only.
__device__ __forceinline__ void axis_eq1(int c, double v, double theta, double& psi, double& chi) {
  const double v2 = v * v;
  const double a0 = 0.5 * v2;
  const double a1 = theta * v + 0.5 * v2 * v;
  const double a2 = theta * theta + 2.5 * theta * v2 + 0.5 * v2 * v2;
  if (c == 0) {
    psi = 1.0 - theta - v2;
    chi = a0 - a2;
  } else {
    psi = 0.5 * (theta + v2 + c * v);
    chi = 0.5 * (a2 + c * a1);
  }
}

}  // namespace lbm
