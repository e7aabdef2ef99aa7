"""Isothermal scheme: Eq. (LBM_f) of Sec. II C at reference temperature theta = varsigma^2 =
1/3 (so Phi = 0), g not evolved (the isothermal mode used for the Poiseuille runs of
Sec. III A), with an optional uniform body force F per unit volume.

One time step is collide-then-stream, literally:
    rho = sum f, rho u = sum c f + F/2                              (moments, Sec. II C)
    f~_i(x, t)       = f_i + 2 beta (f_i^eq - f_i) + (1 - beta)(f_i^* - f_i^eq)   (collide)
    f_i(x + c_i, t+1) = f~_i(x, t)                                   (stream, np.roll)
where f^* is the shifted equilibrium at u* = u + F/rho and theta* = theta (Sec. II C; no heat
source, and alpha = 0 has no effect at constant theta); without a force f^* = f^eq.
with beta = dt / (2 tau + dt) (Sec. II B). In lattice units dt = 1; the relaxation rate is
omega = 2 beta = 1 / tau_LB with tau_LB = tau + 1/2, so that the shear viscosity of
Sec. II D, mu = (1/(2 beta) - 1/2) P dt, gives nu = mu / rho = varsigma^2 (tau_LB - 1/2).

Walls (optional, y direction): half-way bounce-back (Sec. III A, Poiseuille flow), wall
half a spacing outside the first and last rows: a population that would leave the domain
returns to its node with the opposite velocity.
"""
import numpy as np

from .equilibrium import feq, fstar, moments
from .lattice import VARSIGMA2, opposite, velocities


def omega_from_tau_lb(tau_lb):
    """omega = 2 beta = 1/tau_LB; beta = dt/(2 tau + dt) with tau = tau_LB - dt/2 (Sec. II B)."""
    beta = 1.0 / (2.0 * (tau_lb - 0.5) + 1.0)
    return 2.0 * beta


def init_equilibrium(rho, u):
    """Fig. 1: populations initialised to the local equilibrium of the initial fields."""
    return feq(rho, u, VARSIGMA2)


def collide(f, omega, F=None):
    """Post-collision populations f + omega (f^eq - f) + (1 - omega/2)(f^* - f^eq), theta = 1/3."""
    rho, u = moments(f, F=F)
    fe = feq(rho, u, VARSIGMA2)
    out = f + omega * (fe - f)
    if F is not None:
        D = u.shape[0]
        ustar = u + np.asarray(F, dtype=np.float64).reshape((D,) + (1,) * (u.ndim - 1)) / rho
        fs = fstar(rho, ustar, VARSIGMA2, np.zeros_like(ustar))
        out = out + (1.0 - 0.5 * omega) * (fs - fe)
    return out


def stream(ft, walls_y=False):
    """f_i(x + c_i) <- f~_i(x); periodic wrap, or half-way bounce-back at the y walls."""
    Q = ft.shape[0]
    D = {9: 2, 27: 3}[Q]
    c = velocities(D)
    out = np.empty_like(ft)
    for i in range(Q):
        shifted = ft[i]
        for a in range(D):
            if c[i, a]:
                shifted = np.roll(shifted, int(c[i, a]), axis=ft.ndim - 2 - a)
        out[i] = shifted
    if walls_y:
        opp = opposite(D)
        yaxis = ft.ndim - 3  # axis of y within one population plane: (.., y, x)
        for i in range(Q):
            cy = c[i, 1]
            if cy == 0:
                continue
            # rows that received a wrapped value: y = 0 for c_y = +1, y = ny-1 for c_y = -1
            row = 0 if cy > 0 else ft.shape[-2] - 1
            idx = [slice(None)] * (ft.ndim - 1)
            idx[yaxis] = row
            idx = tuple(idx)
            out[i][idx] = ft[opp[i]][idx]
    return out


def run(f, omega, nsteps, walls_y=False, F=None):
    """nsteps repetitions of collide then stream; returns the pre-collision state."""
    for _ in range(nsteps):
        f = stream(collide(f, omega, F), walls_y)
    return f
