"""Double-distribution scheme for an ideal gas, Sec. II C with Fig. 1 and Sec. III A.

Per node and step, in the order of Fig. 1, with an optional uniform body force F (per unit
volume) and heat source Q (energy per unit volume and time); dt = 1:
  rho = sum f,  rho u = sum c f + F/2,  rho E = sum g + (u.F + Q)/2   (Sec. II C moments)
  T = (E - u^2/2) / c_v,  P = rho R T                               (Sec. III A, ideal gas)
  theta = P / rho                                                   (Sec. II A closure)
  u* = u + F/rho                                                    (shifted velocity)
  theta* = theta + alpha theta div u + (gamma - 1) Q/rho with alpha = 0, which the bulk
        viscosity eta = mu (2/D - R/c_v) of Sec. II E gives, and gamma - 1 = R/c_v for the
        ideal gas (Sec. II A, gamma = 1 + (dP/dT)_rho / (rho c_v))
  T* = T + Q/(rho c_v) - F.F/(2 rho^2 c_v)                          (shifted temperature)
  Phi_aa = -(1/rho) d_a (rho u_a^3 + 3 rho u_a (theta - varsigma^2))  (Galilean correction,
        from the unshifted fields)
  f^eq = rho prod Psi(u, theta + u^2),  f* = rho prod Psi(u*, theta* + u*^2 + Phi)   (Sec. II C)
  g^eq = g^eq(rho, u, T, theta),  g* = g^eq(rho, u*, T*, theta*) + q^c term; for the ideal
       gas at Prandtl number 1 (k = mu c_p) the flux q^c = dt P (grad h - (k/mu) grad T)
       vanishes identically because h = c_p T
  tau = mu / P,  beta = dt / (2 tau + dt)                            (Sec. II A, II B)
  f~ = f + 2 beta (f^eq - f) + (1 - beta)(f* - f^eq)                   (Eq. LBM_f)
  g~ = g + 2 beta (g^eq - g) + (1 - beta)(g* - g^eq)                   (Eq. LBM_g)
  stream both (periodic in x, half-way bounce-back at the y walls when enabled).
Without sources (F = 0, Q = 0) u* = u, theta* = theta, T* = T and g* = g^eq.

Derivative inside the Galilean correction. The paper computes all derivatives with standard
second-order central differences, except the first derivative of the correction, for which it
names an upwind-biased scheme without giving the stencil (Sec. II E). Two readings exist here:
  stencil="central"  (p_{i+1} - p_{i-1}) / 2 -- the default, see below;
  stencil="upwind"   second-order one-sided difference keyed on the sign of u_a at the node,
                     (3 p_i - 4 p_{i-1} + p_{i-2})/2 for u_a > 0, -(3 p_i - 4 p_{i+1} + p_{i+2})/2
                     for u_a < 0, central for u_a = 0.
Both are second order. The one-sided reading switches sides wherever u_a changes sign; in a
shear layer the transverse velocity is near zero with a noisy sign, and that switching makes
the thermal shear layer with walls blow up within a few hundred steps (first- and third-order
sign-keyed variants behave the same), while the central stencil stays stable. Ghost rows at a
wall use zero-order extrapolation of the nearest fluid row (the paper's default extrapolation
for unspecified boundary data, Sec. III A, Rayleigh flow).
"""
import numpy as np

from . import bgk
from .equilibrium import feq, fstar, geq
from .lattice import VARSIGMA2, velocities


class Gas:
    """Ideal-gas parameters: gas constant R, heat capacity c_v, dynamic viscosity mu."""

    def __init__(self, R, cv, mu):
        self.R = float(R)
        self.cv = float(cv)
        self.mu = float(mu)

    @property
    def gamma(self):
        """gamma = 1 + (dP/dT)_rho / (rho c_v) with P = rho R T: 1 + R/c_v = c_p/c_v."""
        return 1.0 + self.R / self.cv


def _field(F, D, shape):
    """The force as a (D,) + node-shape array (zero when F is None)."""
    if F is None:
        return np.zeros((D,) + shape)
    F = np.asarray(F, dtype=np.float64)
    if F.ndim == 1:  # one vector for every node
        F = F.reshape((D,) + (1,) * len(shape))
    return np.broadcast_to(F, (D,) + shape)


def closure(rho, u, rhoE, gas):
    """T, P, theta from the conserved fields (ideal gas, Sec. III A)."""
    E = rhoE / rho
    usq = (u * u).sum(axis=0)
    T = (E - 0.5 * usq) / gas.cv
    P = rho * gas.R * T
    theta = P / rho
    return T, P, theta


def _shifted(p, axis, wall):
    pad = [(0, 0)] * p.ndim
    pad[axis] = (2, 2)
    q = np.pad(p, pad, mode="edge" if wall else "wrap")
    n = p.shape[axis]

    def sl(k):
        idx = [slice(None)] * p.ndim
        idx[axis] = slice(2 + k, 2 + k + n)
        return q[tuple(idx)]

    return sl


def central_derivative(p, axis, wall):
    """(p_{i+1} - p_{i-1}) / 2 along `axis`, periodic or with extrapolated wall ghosts."""
    sl = _shifted(p, axis, wall)
    return 0.5 * (sl(1) - sl(-1))


def upwind_derivative(p, u_a, axis, wall):
    """Second-order one-sided difference on the upwind side of u_a (central where u_a = 0)."""
    sl = _shifted(p, axis, wall)
    back = 0.5 * (3.0 * sl(0) - 4.0 * sl(-1) + sl(-2))
    fwd = -0.5 * (3.0 * sl(0) - 4.0 * sl(1) + sl(2))
    cen = 0.5 * (sl(1) - sl(-1))
    return np.where(u_a > 0, back, np.where(u_a < 0, fwd, cen))


def galilean_correction(rho, u, theta, walls_y, stencil="central"):
    """dt Phi_aa = -(1/rho) d_a (rho u_a^3 + 3 rho u_a (theta - varsigma^2)), per axis."""
    D = u.shape[0]
    out = np.empty_like(u)
    for a in range(D):
        phi = rho * u[a] ** 3 + 3.0 * rho * u[a] * (theta - VARSIGMA2)
        axis = rho.ndim - 1 - a
        wall = walls_y and a == 1
        if stencil == "central":
            d = central_derivative(phi, axis, wall)
        elif stencil == "upwind":
            d = upwind_derivative(phi, u[a], axis, wall)
        else:
            raise ValueError(stencil)
        out[a] = -d / rho
    return out


def equilibria(rho, u, rhoE, gas, walls_y, phi_on=True, stencil="central", F=None, Q=0.0):
    """f^eq, f*, g^eq, g*, beta at every node (Fig. 1 order) from the moments (rho, u, rho E
    already carry the half-step source terms)."""
    D = u.shape[0]
    T, P, theta = closure(rho, u, rhoE, gas)
    e = gas.cv * T
    Fv = _field(F, D, rho.shape)
    ustar = u + Fv / rho
    thetastar = theta + (gas.gamma - 1.0) * Q / rho
    Tstar = T + Q / (rho * gas.cv) - (Fv * Fv).sum(axis=0) / (2.0 * rho * rho * gas.cv)
    fe = feq(rho, u, theta)
    Phi = galilean_correction(rho, u, theta, walls_y, stencil) if phi_on else np.zeros_like(u)
    fs = fstar(rho, ustar, thetastar, Phi)
    ge = geq(rho, u, theta, e)
    gs = geq(rho, ustar, thetastar, gas.cv * Tstar)
    tau = gas.mu / P
    beta = 1.0 / (2.0 * tau + 1.0)
    return fe, fs, ge, gs, beta


def moments(f, g, F=None, Q=0.0):
    """rho = sum f, rho u = sum c f + F/2, rho E = sum g + (u.F + Q)/2 (Sec. II C)."""
    D = {9: 2, 27: 3}[f.shape[0]]
    c = velocities(D).astype(np.float64)
    rho = f.sum(axis=0)
    Fv = _field(F, D, rho.shape)
    u = (np.stack([np.tensordot(c[:, a], f, axes=(0, 0)) for a in range(D)]) + 0.5 * Fv) / rho
    return rho, u, g.sum(axis=0) + 0.5 * ((u * Fv).sum(axis=0) + Q)


def init_equilibrium(rho, u, T, gas):
    """Fig. 1: f <- f^eq, g <- g^eq of the initial fields."""
    theta = gas.R * T
    return feq(rho, u, theta), geq(rho, u, theta, gas.cv * T)


def collide(f, g, gas, walls_y, phi_on=True, stencil="central", F=None, Q=0.0):
    rho, u, rhoE = moments(f, g, F, Q)
    fe, fs, ge, gs, beta = equilibria(rho, u, rhoE, gas, walls_y, phi_on, stencil, F, Q)
    ft = f + 2.0 * beta * (fe - f) + (1.0 - beta) * (fs - fe)
    gt = g + 2.0 * beta * (ge - g) + (1.0 - beta) * (gs - ge)
    return ft, gt


def run(f, g, gas, nsteps, walls_y=True, phi_on=True, stencil="central", F=None, Q=0.0):
    for _ in range(nsteps):
        ft, gt = collide(f, g, gas, walls_y, phi_on, stencil, F, Q)
        f = bgk.stream(ft, walls_y)
        g = bgk.stream(gt, walls_y)
    return f, g


def temperature(f, g, gas, F=None, Q=0.0):
    rho, u, rhoE = moments(f, g, F, Q)
    T, _, _ = closure(rho, u, rhoE, gas)
    return rho, u, T
