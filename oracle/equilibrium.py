"""Product-form equilibria, Sec. II C.

psi       the two-variable functions Psi_ia(xi_a, zeta_aa) = 1 - c_ia^2
          + 1/2 [(3 c_ia^2 - 2) zeta_aa + c_ia xi_a]
feq       f_i^eq = rho prod_a Psi_ia(u_a, theta + u_a^2)        (local equilibrium)
fstar     f_i^* = rho prod_a Psi_ia(u*_a, theta* + u*_a^2 + dt Phi_aa)   (shifted equilibrium)
geq       g_i^eq = rho prod_a Psi_ia(O_a, O_a^2) E, with the operators
          O_a(theta) E = theta dE/du_a + u_a E acting on the generating function
          E = e + u^2/2; computed here literally, by applying the operator polynomial
          to E written as a polynomial in the velocity components and evaluating it.

All functions are float64 and vectorised over nodes: rho, theta, e have node shape S,
u has shape (D,) + S, the populations have shape (Q,) + S.
"""
import numpy as np

from .lattice import velocities


def psi(c, xi, zeta):
    """Psi(xi, zeta) for one velocity component c in {-1, 0, 1} (Sec. II C)."""
    return 1.0 - c * c + 0.5 * ((3 * c * c - 2) * zeta + c * xi)


def feq(rho, u, theta):
    """Local equilibrium f_i^eq = rho prod_a Psi_ia(u_a, theta + u_a^2)."""
    u = np.asarray(u, dtype=np.float64)
    D = u.shape[0]
    c = velocities(D)
    out = np.empty((len(c),) + np.shape(rho), dtype=np.float64)
    for i, ci in enumerate(c):
        prod = np.asarray(rho, dtype=np.float64)
        for a in range(D):
            prod = prod * psi(ci[a], u[a], theta + u[a] * u[a])
        out[i] = prod
    return out


def fstar(rho, ustar, thetastar, Phi):
    """Shifted equilibrium f_i^* = rho prod_a Psi_ia(u*_a, theta* + u*_a^2 + Phi_aa).

    Phi holds dt * Phi_aa per axis, shape (D,) + S (dt = 1 in lattice units).
    """
    ustar = np.asarray(ustar, dtype=np.float64)
    D = ustar.shape[0]
    c = velocities(D)
    out = np.empty((len(c),) + np.shape(rho), dtype=np.float64)
    for i, ci in enumerate(c):
        prod = np.asarray(rho, dtype=np.float64)
        for a in range(D):
            prod = prod * psi(ci[a], ustar[a], thetastar + ustar[a] * ustar[a] + Phi[a])
        out[i] = prod
    return out


# --- operator-generated energy equilibrium -------------------------------------------
# A polynomial in the formal velocity variables U_1..U_D is a dict mapping the exponent
# tuple (p_1, .., p_D) to a coefficient (scalar or per-node array).

def _poly_add(acc, poly, scale):
    for p, coef in poly.items():
        acc[p] = acc.get(p, 0.0) + scale * coef
    return acc


def _apply_O(poly, a, theta):
    """O_a(theta) P = theta dP/dU_a + U_a P."""
    out = {}
    for p, coef in poly.items():
        if p[a] > 0:
            q = list(p)
            q[a] -= 1
            q = tuple(q)
            out[q] = out.get(q, 0.0) + theta * p[a] * coef
        q = list(p)
        q[a] += 1
        q = tuple(q)
        out[q] = out.get(q, 0.0) + coef
    return out


def _apply_psi_operator(poly, c, a, theta):
    """Psi_ia(O_a, O_a^2) P = (1 - c^2) P + 1/2 (3c^2 - 2) O_a^2 P + 1/2 c O_a P."""
    o1 = _apply_O(poly, a, theta)
    o2 = _apply_O(o1, a, theta)
    out = {}
    _poly_add(out, poly, 1.0 - c * c)
    _poly_add(out, o2, 0.5 * (3 * c * c - 2))
    _poly_add(out, o1, 0.5 * c)
    return out


def _evaluate(poly, u):
    total = 0.0
    for p, coef in poly.items():
        term = coef
        for a, pa in enumerate(p):
            if pa:
                term = term * u[a] ** pa
        total = total + term
    return total


def energy_generating_polynomial(e, D):
    """E = e + sum_a U_a^2 / 2 as a polynomial (Sec. II C, generating function)."""
    zero = (0,) * D
    poly = {zero: np.asarray(e, dtype=np.float64)}
    for a in range(D):
        p = [0] * D
        p[a] = 2
        poly[tuple(p)] = 0.5
    return poly


def geq(rho, u, theta, e):
    """g_i^eq = rho prod_a Psi_ia(O_a(theta), O_a(theta)^2) E, evaluated at U = u."""
    u = np.asarray(u, dtype=np.float64)
    D = u.shape[0]
    c = velocities(D)
    E = energy_generating_polynomial(e, D)
    out = np.empty((len(c),) + np.shape(rho), dtype=np.float64)
    for i, ci in enumerate(c):
        poly = E
        for a in range(D):
            poly = _apply_psi_operator(poly, int(ci[a]), a, theta)
        out[i] = np.asarray(rho, dtype=np.float64) * _evaluate(poly, u)
    return out


def moments(f, g=None, F=None):
    """Conserved fields (Sec. II C, definitions of rho, rho u, rho E): rho = sum f and
    rho u = sum c f + dt F / 2 (dt = 1; F = 0 when not given; a uniform F has shape (D,)).

    Returns rho, u (shape (D,) + S) and, if g is given, rho E = sum g (no heat source, and
    the u . F / 2 term is left to the caller that evolves g with a force).
    """
    Q = f.shape[0]
    D = {9: 2, 27: 3}[Q]
    c = velocities(D)
    rho = f.sum(axis=0)
    j = np.stack([np.tensordot(c[:, a].astype(np.float64), f, axes=(0, 0)) for a in range(D)])
    if F is not None:
        j = j + 0.5 * np.asarray(F, dtype=np.float64).reshape((D,) + (1,) * (j.ndim - 1))
    u = j / rho
    if g is None:
        return rho, u
    return rho, u, g.sum(axis=0)
