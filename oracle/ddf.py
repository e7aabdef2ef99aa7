"""Double-distribution scheme for an ideal gas, Sec. II C with Fig. 1 and Sec. III A.

Per node and step, in the order of Fig. 1, with an optional uniform body force F (per unit
volume) and heat source Q (energy per unit volume and time); dt = 1:
  rho = sum f,  rho u = sum c f + F/2,  rho E = sum g + (u.F + Q)/2   (Sec. II C moments)
  T = (E - u^2/2) / c_v,  P = rho R T                               (Sec. III A, ideal gas)
  theta = P / rho                                                   (Sec. II A closure)
  u* = u + F/rho                                                    (shifted velocity)
  theta* = theta + alpha theta div u + (gamma - 1) Q/rho with
        alpha = (D+2)/D - gamma - eta/mu (Sec. II A; 0 for the Navier-Stokes bulk viscosity
        eta = mu (2/D - R/c_v) of Sec. II E, the default) and gamma - 1 = R/c_v for the
        ideal gas (gamma = 1 + (dP/dT)_rho / (rho c_v)); div u by central differences
  T* = T + Q/(rho c_v) - F.F/(2 rho^2 c_v)                          (shifted temperature)
  Phi_aa = -(1/rho) d_a (rho u_a^3 + 3 rho u_a (theta - varsigma^2))  (Galilean correction,
        from the unshifted fields)
  f^eq = rho prod Psi(u, theta + u^2),  f* = rho prod Psi(u*, theta* + u*^2 + Phi)   (Sec. II C)
  g^eq = g^eq(rho, u, T, theta),  g* = g^eq(rho, u*, T*, theta*) + c_i.q^c/2 on |c_i|^2 = 1,
       q^c = dt P (grad h - (k/mu) grad T) = P (c_p - k/mu) grad T for the ideal gas
       (h = c_p T), k = mu c_p / Pr; it vanishes at Prandtl number 1 (the default); grad T by
       central differences
  tau = mu / P,  beta = dt / (2 tau + dt)                            (Sec. II A, II B)
  f~ = f + 2 beta (f^eq - f) + (1 - beta)(f* - f^eq)                   (Eq. LBM_f)
  g~ = g + 2 beta (g^eq - g) + (1 - beta)(g* - g^eq)                   (Eq. LBM_g)
  stream both (periodic in x, half-way bounce-back at the y walls when enabled).
Without sources (F = 0, Q = 0) at Pr = 1 and the Navier-Stokes bulk viscosity u* = u,
theta* = theta, T* = T and g* = g^eq.

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
for unspecified boundary data, Sec. III A, Rayleigh flow). On the boundary nodes of the
non-equilibrium extrapolation walls the side is keyed on the wall velocity (upwind_key).
"""
import numpy as np

from . import bgk
from .equilibrium import feq, fstar, geq
from .lattice import VARSIGMA2, velocities


class Gas:
    """Fluid parameters: gas constant R, heat capacity c_v, dynamic viscosity mu, Prandtl
    number Pr = mu c_p0 / k (thermal conductivity k, c_p0 = c_v + R) and bulk viscosity ratio
    eta/mu (None: the Navier-Stokes value 2/D - R/c_v named in Sec. II E, for which alpha = 0 in
    the ideal gas). a, b: van der Waals constants (Sec. III C, Eq. vdw_eos),
    P = rho R T / (1 - b rho) - a rho^2 with e = c_v T - a rho (Eq. lbm_temp); a = b = 0 is
    the ideal gas of Sec. III A."""

    def __init__(self, R, cv, mu, prandtl=1.0, eta_over_mu=None, a=0.0, b=0.0):
        self.R = float(R)
        self.cv = float(cv)
        self.mu = float(mu)
        self.prandtl = float(prandtl)
        self.eta_over_mu = None if eta_over_mu is None else float(eta_over_mu)
        self.a = float(a)
        self.b = float(b)

    @property
    def ideal(self):
        return self.a == 0.0 and self.b == 0.0

    # ---- equation of state (van der Waals; ideal gas at a = b = 0) ----------------------
    def pressure(self, rho, T):
        if self.ideal:
            return rho * self.R * T
        return rho * self.R * T / (1.0 - self.b * rho) - self.a * rho * rho

    def temperature_of(self, rho, e):
        """T from the specific internal energy (Eq. lbm_temp: T = (e + a rho) / c_v)."""
        if self.ideal:
            return e / self.cv
        return (e + self.a * rho) / self.cv

    def internal_energy(self, rho, T):
        if self.ideal:
            return self.cv * T
        return self.cv * T - self.a * rho

    def gamma_minus_1(self, rho):
        """(dP/dT)_rho / (rho c_v) (Sec. II A, Eq. corr_heat_source); R / c_v for the ideal gas."""
        if self.ideal:
            return self.gamma - 1.0
        return self.R / ((1.0 - self.b * rho) * self.cv)

    def sound_speed2(self, rho, T):
        """c_s^2 = (dP/drho)_T + T / (rho^2 c_v) (dP/dT)_rho^2 (Sec. II A)."""
        dPdrho = self.R * T / (1.0 - self.b * rho) ** 2 - 2.0 * self.a * rho
        dPdT = rho * self.R / (1.0 - self.b * rho)
        return dPdrho + T / (rho * rho * self.cv) * dPdT * dPdT

    def alpha_field(self, D, rho, T, P):
        """alpha = (D+2)/D - rho c_s^2 / P - eta/mu (Eq. corr_bulk) per node; for the ideal gas
        the constant of alpha()."""
        if self.ideal:
            return self.alpha(D)
        eta = (2.0 / D - self.R / self.cv) if self.eta_over_mu is None else self.eta_over_mu
        return (D + 2.0) / D - rho * self.sound_speed2(rho, T) / P - eta

    @property
    def gamma(self):
        """gamma = 1 + (dP/dT)_rho / (rho c_v) with P = rho R T: 1 + R/c_v = c_p/c_v."""
        return 1.0 + self.R / self.cv

    @property
    def cp(self):
        return self.cv + self.R

    def alpha(self, D):
        """alpha = (D+2)/D - rho c_s^2/P - eta/mu (Sec. II A) with rho c_s^2 / P = gamma for the
        ideal gas; exactly 0 for the Navier-Stokes bulk viscosity."""
        if self.eta_over_mu is None:
            return 0.0
        return (D + 2.0) / D - self.gamma - self.eta_over_mu

    def qc_coefficient(self):
        """q^c = dt P (grad h - (k/mu) grad T) (Eq. qc_1) with h = e + P/rho = c_p T for the
        ideal gas, so grad h = c_p grad T for any linear difference operator and
        q^c = P (c_p - k/mu) grad T, k/mu = c_p / Pr; exactly 0 at Pr = 1."""
        return self.cp - self.cp / self.prandtl


def _field(F, D, shape):
    """The force as a (D,) + node-shape array (zero when F is None)."""
    if F is None:
        return np.zeros((D,) + shape)
    F = np.asarray(F, dtype=np.float64)
    if F.ndim == 1:  # one vector for every node
        F = F.reshape((D,) + (1,) * len(shape))
    return np.broadcast_to(F, (D,) + shape)


def closure(rho, u, rhoE, gas):
    """T, P, theta from the conserved fields: T from the caloric relation (Sec. III A ideal gas,
    Eq. lbm_temp for van der Waals), P from the equation of state, theta = P / rho."""
    E = rhoE / rho
    usq = (u * u).sum(axis=0)
    T = gas.temperature_of(rho, E - 0.5 * usq)
    P = gas.pressure(rho, T)
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


def divergence(u, walls_y):
    """div u by second-order central differences (Sec. II E), wall ghosts as for Phi."""
    D = u.shape[0]
    return sum(central_derivative(u[a], u.ndim - 2 - a, walls_y and a == 1) for a in range(D))


def galilean_correction(rho, u, theta, walls_y, stencil="central", key=None):
    """dt Phi_aa = -(1/rho) d_a (rho u_a^3 + 3 rho u_a (theta - varsigma^2)), per axis.
    key: the velocity whose sign picks the upwind side (default u; see upwind_key)."""
    D = u.shape[0]
    key = u if key is None else key
    out = np.empty_like(u)
    for a in range(D):
        phi = rho * u[a] ** 3 + 3.0 * rho * u[a] * (theta - VARSIGMA2)
        axis = rho.ndim - 1 - a
        wall = walls_y and a == 1
        if stencil == "central":
            d = central_derivative(phi, axis, wall)
        elif stencil == "upwind":
            d = upwind_derivative(phi, key[a], axis, wall)
        else:
            raise ValueError(stencil)
        out[a] = -d / rho
    return out


def upwind_key(u, neq):
    """Velocity that picks the upwind side of the Phi derivative. On the boundary nodes of the
    non-equilibrium extrapolation walls (rows or planes y = 0 and ny - 1) it is the wall
    velocity: there the fluid velocity equals it up to rounding, and the sign of a component
    that vanishes (the normal one, or a zero tangential one) is rounding noise, so the y
    derivative on those rows is central and the tangential ones follow the wall's motion.
    Everywhere else, and without such walls, it is u itself."""
    if neq is None:
        return u
    key = u.copy()
    ny = u.shape[-2]
    for side, row in enumerate((0, ny - 1)):
        for a in range(u.shape[0]):
            key[a][..., row, :] = neq.u[side][a]
    return key


def equilibria(rho, u, rhoE, gas, walls_y, phi_on=True, stencil="central", F=None, Q=0.0,
               neq=None):
    """f^eq, f*, g^eq, g*, beta at every node (Fig. 1 order) from the moments (rho, u, rho E
    already carry the half-step source terms); neq (NeqWalls) only keys the upwind side on
    the boundary nodes (upwind_key)."""
    D = u.shape[0]
    T, P, theta = closure(rho, u, rhoE, gas)
    e = gas.internal_energy(rho, T)
    Fv = _field(F, D, rho.shape)
    ustar = u + Fv / rho
    thetastar = theta + gas.gamma_minus_1(rho) * Q / rho
    alpha = gas.alpha_field(D, rho, T, P)
    if np.any(alpha != 0.0):  # theta* = theta + dt alpha theta div u + ... (Eq. sh_temp_1)
        thetastar = thetastar + alpha * theta * divergence(u, walls_y)
    Tstar = T + Q / (rho * gas.cv) - (Fv * Fv).sum(axis=0) / (2.0 * rho * rho * gas.cv)
    fe = feq(rho, u, theta)
    Phi = (galilean_correction(rho, u, theta, walls_y, stencil, upwind_key(u, neq)) if phi_on
           else np.zeros_like(u))
    fs = fstar(rho, ustar, thetastar, Phi)
    ge = geq(rho, u, theta, e)
    gs = geq(rho, ustar, thetastar, gas.internal_energy(rho, Tstar))
    c = velocities(D)
    qc = None
    if gas.ideal:
        kq = gas.qc_coefficient()
        if kq != 0.0:
            qc = [P * kq * central_derivative(T, rho.ndim - 1 - a, walls_y and a == 1)
                  for a in range(D)]
    else:  # q^c = dt P (grad h - (k/mu) grad T), h = e + P/rho (Eqs. qc_1, enthalpy)
        h = e + P / rho
        kmu = gas.cp / gas.prandtl
        qc = [P * (central_derivative(h, rho.ndim - 1 - a, walls_y and a == 1)
                   - kmu * central_derivative(T, rho.ndim - 1 - a, walls_y and a == 1))
              for a in range(D)]
    if qc is not None:  # g* += c_i . q^c / 2 on the velocities with |c_i|^2 = 1 (Eq. LBMgstar)
        for i, ci in enumerate(c):
            if (ci * ci).sum() == 1:
                gs[i] = gs[i] + 0.5 * sum(ci[a] * qc[a] for a in range(D))
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
    theta = gas.pressure(rho, T) / rho
    return feq(rho, u, theta), geq(rho, u, theta, gas.internal_energy(rho, T))


def collide(f, g, gas, walls_y, phi_on=True, stencil="central", F=None, Q=0.0, neq=None):
    rho, u, rhoE = moments(f, g, F, Q)
    fe, fs, ge, gs, beta = equilibria(rho, u, rhoE, gas, walls_y, phi_on, stencil, F, Q, neq)
    ft = f + 2.0 * beta * (fe - f) + (1.0 - beta) * (fs - fe)
    gt = g + 2.0 * beta * (ge - g) + (1.0 - beta) * (gs - ge)
    return ft, gt


class NeqWalls:
    """Non-equilibrium extrapolation walls (App. B, thermal Couette): the first and last rows
    (D2Q9) or planes (D3Q27) y = 0 and y = ny - 1 are boundary nodes B on the walls, with wall
    velocities u_lo, u_hi (D components) and temperatures T_lo, T_hi; N is the neighbouring row
    or plane (1 or ny - 2).
    density="pressure" (the default reading) takes the rho_B that continues the neighbour's
    pressure to the wall, P(rho_B, T_W) = P(rho_N, T_N): rho_N T_N / T_W for the ideal gas, the
    root of the van der Waals isotherm (wall_density_vdw) otherwise; density="literal" takes
    rho_B = rho_N, the paper's extrapolation written out (the two agree where T_N = T_W)."""

    def __init__(self, u_lo, T_lo, u_hi, T_hi, density="pressure"):
        self.u = (np.asarray(u_lo, dtype=np.float64), np.asarray(u_hi, dtype=np.float64))
        self.T = (float(T_lo), float(T_hi))
        if density not in ("pressure", "literal"):
            raise ValueError(density)
        self.density = density


def critical_temperature(gas):
    """T_cr = 8 a / (27 b R) of the van der Waals isotherms (Sec. III C): above it P(rho) is
    strictly increasing on 0 < rho < 1/b."""
    return 8.0 * gas.a / (27.0 * gas.b * gas.R)


def wall_density_vdw(P_N, T_W, gas, iters=200):
    """rho_B with P(rho_B, T_W) = P_N on a supercritical van der Waals isotherm (T_W > T_cr,
    b > 0), by bisection on (0, 1/b) where P is strictly increasing; run until the bracket
    stops shrinking (float64 resolution)."""
    if not (gas.b > 0.0 and T_W > critical_temperature(gas)):
        raise ValueError("the pressure-continued wall density needs b > 0 and T_W > T_cr")
    lo = np.zeros_like(P_N)
    hi = np.full_like(P_N, 1.0 / gas.b)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        above = gas.pressure(mid, T_W) > P_N
        hi = np.where(above, mid, hi)
        lo = np.where(above, lo, mid)
    return 0.5 * (lo + hi)


def apply_neq_walls(f, g, gas, walls):
    """Boundary rows of the pre-collision populations:
    f_B = f^eq(rho_B, u_W, T_W) + (f_N - f^eq(rho_N, u_N, T_N)), and the same for g (App. B),
    with rho_B from NeqWalls.density; the wall equilibria take theta_W = P(rho_B, T_W)/rho_B
    and e_W = e(rho_B, T_W) of the fluid's equation of state (R T_W and c_v T_W for the ideal
    gas). No sources (the context rejects them with these walls)."""
    rho, u, rhoE = moments(f, g)
    T, _, theta = closure(rho, u, rhoE, gas)
    fe = feq(rho, u, theta)
    ge = geq(rho, u, theta, gas.internal_energy(rho, T))
    ny = f.shape[-2]
    f, g = f.copy(), g.copy()
    D = u.shape[0]
    for side, (B, N) in enumerate(((0, 1), (ny - 1, ny - 2))):
        TW = walls.T[side]
        rN, TN = rho[..., N, :], T[..., N, :]
        if walls.density == "literal":
            rB = rN
        elif gas.ideal:
            rB = rN * TN / TW
        else:
            rB = wall_density_vdw(gas.pressure(rN, TN), TW, gas)
        uW = walls.u[side].reshape((D,) + (1,) * rB.ndim) * np.ones((D,) + rB.shape)
        TWf = np.full(rB.shape, TW)
        thetaW = gas.R * TWf if gas.ideal else gas.pressure(rB, TWf) / rB
        eW = gas.internal_energy(rB, TWf)
        f[..., B, :] = feq(rB, uW, thetaW) + (f[..., N, :] - fe[..., N, :])
        g[..., B, :] = geq(rB, uW, thetaW, eW) + (g[..., N, :] - ge[..., N, :])
    return f, g


def run(f, g, gas, nsteps, walls_y=True, phi_on=True, stencil="central", F=None, Q=0.0,
        neq=None):
    """nsteps of collide-then-stream from the pre-collision state (f, g). With neq (NeqWalls)
    the boundary rows are rebuilt before every collision and once more at the end, so the
    returned state is the pre-collision state of the last time; streaming then wraps
    periodically (the wrapped boundary rows are rebuilt) and derivative ghosts at the walls
    are zero-order as for the bounce-back walls."""
    if neq is not None:
        for _ in range(nsteps):
            f, g = apply_neq_walls(f, g, gas, neq)
            ft, gt = collide(f, g, gas, True, phi_on, stencil, F, Q, neq)
            f, g = bgk.stream(ft), bgk.stream(gt)
        return apply_neq_walls(f, g, gas, neq)
    for _ in range(nsteps):
        ft, gt = collide(f, g, gas, walls_y, phi_on, stencil, F, Q)
        f = bgk.stream(ft, walls_y)
        g = bgk.stream(gt, walls_y)
    return f, g


def temperature(f, g, gas, F=None, Q=0.0):
    rho, u, rhoE = moments(f, g, F, Q)
    T, _, _ = closure(rho, u, rhoE, gas)
    return rho, u, T
