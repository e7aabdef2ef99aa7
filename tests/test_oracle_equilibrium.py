"""Pins of the oracle's lattice and equilibria against what the paper and mathematics fix."""
import numpy as np
import pytest

from oracle import equilibrium as eq
from oracle.lattice import VARSIGMA2, all_velocity_tuples, opposite, velocities


@pytest.mark.parametrize("D", [2, 3])
def test_velocity_set_is_nearest_neighbour_lattice(D):
    c = velocities(D)
    assert len(c) == 3 ** D
    assert {tuple(int(v) for v in ci) for ci in c} == all_velocity_tuples(D)
    # the ordering puts -c_i at Q-1-i
    assert np.array_equal(opposite(D), np.arange(3 ** D)[::-1])


def test_rest_weights_d2q9_textbook():
    # u = 0, theta = 1/3 gives the standard D2Q9 weights 4/9, 1/9, 1/36
    f = eq.feq(np.array(1.0), np.zeros(2), VARSIGMA2)
    c = velocities(2)
    for i, ci in enumerate(c):
        n = int(np.abs(ci).sum())
        assert f[i] == pytest.approx({0: 4 / 9, 1: 1 / 9, 2: 1 / 36}[n], rel=1e-15)


def test_rest_weights_d3q27_textbook():
    f = eq.feq(np.array(1.0), np.zeros(3), VARSIGMA2)
    c = velocities(3)
    for i, ci in enumerate(c):
        n = int(np.abs(ci).sum())
        assert f[i] == pytest.approx({0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}[n], rel=1e-15)


def _random_state(D, shape, seed, theta_fixed=None):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 2.0, size=shape)
    u = rng.uniform(-0.2, 0.2, size=(D,) + shape)
    theta = rng.uniform(0.2, 0.5, size=shape) if theta_fixed is None else theta_fixed
    return rho, u, theta


@pytest.mark.parametrize("D", [2, 3])
def test_feq_moments_match_product_form_identities(D):
    # Sec. II C: sum Psi = 1, sum c Psi = xi, sum c^2 Psi = zeta per axis, so the moments of
    # f^eq up to second order per axis factorise.
    rho, u, theta = _random_state(D, (5, 4), seed=1)
    f = eq.feq(rho, u, theta)
    c = velocities(D).astype(np.float64)
    mom = lambda w: np.tensordot(w, f, axes=(0, 0))
    np.testing.assert_allclose(mom(np.ones(len(c))), rho, rtol=1e-14)
    for a in range(D):
        np.testing.assert_allclose(mom(c[:, a]), rho * u[a], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(mom(c[:, a] ** 2), rho * (theta + u[a] ** 2), rtol=1e-13)
        # lattice closure c^3 = c: the third moment is rho u, not rho(u^3 + 3 theta u)
        np.testing.assert_allclose(mom(c[:, a] ** 3), rho * u[a], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(mom(c[:, 0] * c[:, 1]), rho * u[0] * u[1], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(mom(c[:, 0] ** 2 * c[:, 1] ** 2),
                               rho * (theta + u[0] ** 2) * (theta + u[1] ** 2), rtol=1e-13)
    # Maxwellian values of the off-diagonal third-order moment: rho u_x (theta + u_y^2)
    np.testing.assert_allclose(mom(c[:, 0] * c[:, 1] ** 2), rho * u[0] * (theta + u[1] ** 2),
                               rtol=1e-13, atol=1e-15)


def test_d3q27_z_marginal_is_d2q9():
    rho, u2, theta = _random_state(2, (3, 5), seed=2)
    u3 = np.concatenate([u2, np.zeros((1, 3, 5))])
    f3 = eq.feq(rho, u3, theta)
    f2 = eq.feq(rho, u2, theta)
    c3 = velocities(3)
    c2 = velocities(2)
    for j, cj in enumerate(c2):
        mask = (c3[:, 0] == cj[0]) & (c3[:, 1] == cj[1])
        np.testing.assert_allclose(f3[mask].sum(axis=0), f2[j], rtol=1e-14)


def test_fstar_with_zero_shift_is_feq():
    rho, u, theta = _random_state(2, (4,), seed=3)
    np.testing.assert_array_equal(eq.fstar(rho, u, theta, np.zeros_like(u)), eq.feq(rho, u, theta))


def test_fstar_shift_changes_only_the_diagonal_second_moment():
    rho, u, theta = _random_state(2, (6,), seed=4)
    Phi = np.random.default_rng(5).uniform(-1e-2, 1e-2, size=u.shape)
    f = eq.fstar(rho, u, theta, Phi)
    c = velocities(2).astype(np.float64)
    mom = lambda w: np.tensordot(w, f, axes=(0, 0))
    np.testing.assert_allclose(mom(np.ones(9)), rho, rtol=1e-14)
    for a in range(2):
        np.testing.assert_allclose(mom(c[:, a]), rho * u[a], rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(mom(c[:, a] ** 2), rho * (theta + u[a] ** 2 + Phi[a]), rtol=1e-13)


@pytest.mark.parametrize("D", [2, 3])
def test_geq_moments_match_appendix_fluxes(D):
    # Sec. II A: sum g^eq = rho E. App. A: Pi_1(g^(0)) = u (rho E + P) and
    # Pi_2(g^(0)) = u u (rho E + 2P) + (E + P/rho) P I, with theta = P / rho.
    rho, u, theta = _random_state(D, (4, 3), seed=6)
    rng = np.random.default_rng(7)
    e = rng.uniform(0.5, 3.0, size=rho.shape)
    g = eq.geq(rho, u, theta, e)
    c = velocities(D).astype(np.float64)
    mom = lambda w: np.tensordot(w, g, axes=(0, 0))
    E = e + 0.5 * (u * u).sum(axis=0)
    P = rho * theta
    np.testing.assert_allclose(mom(np.ones(len(c))), rho * E, rtol=1e-13)
    for a in range(D):
        np.testing.assert_allclose(mom(c[:, a]), u[a] * (rho * E + P), rtol=1e-12, atol=1e-14)
        for b in range(D):
            expect = u[a] * u[b] * (rho * E + 2 * P) + (a == b) * (E + P / rho) * P
            np.testing.assert_allclose(mom(c[:, a] * c[:, b]), expect, rtol=1e-12, atol=1e-14)


def test_geq_at_rest_is_energy_times_weights_plus_flux_term():
    # u = 0: g_i = rho e w_i + rho [chi_cx(0) psi_cy(0) + psi_cx(0) chi_cy(0)] with chi from
    # the operator algebra evaluated by hand: O E = theta dE/du (0 at u = 0),
    # O^2 (u^2/2) = theta^2 at u = 0, so chi_0 = -theta^2, chi_pm = theta^2/2.
    theta = 0.3
    rho = np.array(1.7)
    e = np.array(2.1)
    g = eq.geq(rho, np.zeros(2), theta, e)
    f = eq.feq(rho, np.zeros(2), theta)
    psi0 = {0: 1 - theta, 1: theta / 2, -1: theta / 2}
    chi0 = {0: -theta ** 2, 1: theta ** 2 / 2, -1: theta ** 2 / 2}
    for i, (cx, cy) in enumerate(velocities(2)):
        expect = e * f[i] + rho * (chi0[cx] * psi0[cy] + psi0[cx] * chi0[cy])
        assert g[i] == pytest.approx(float(expect), rel=1e-14)


def test_geq_closed_form_derivation_matches_operator_application():
    # Independent hand derivation of g^eq for D2Q9:
    # g_i = e f_i + rho [chi_cx(u_x) psi_cy(u_y) + psi_cx(u_x) chi_cy(u_y)],
    # a0 = u^2/2, a1 = theta u + u^3/2, a2 = theta^2 + 5/2 theta u^2 + u^4/2,
    # chi_0 = a0 - a2, chi_pm = (a2 +- a1)/2, psi_c(u) = Psi(c; u, theta + u^2).
    rho, u, theta = _random_state(2, (7,), seed=8)
    e = np.random.default_rng(9).uniform(0.5, 2.0, size=rho.shape)
    g = eq.geq(rho, u, theta, e)

    def psi1(c, v):
        return {0: 1 - theta - v * v, 1: 0.5 * (theta + v * v + v), -1: 0.5 * (theta + v * v - v)}[c]

    def chi(c, v):
        a0 = 0.5 * v * v
        a1 = theta * v + 0.5 * v ** 3
        a2 = theta ** 2 + 2.5 * theta * v * v + 0.5 * v ** 4
        return {0: a0 - a2, 1: 0.5 * (a2 + a1), -1: 0.5 * (a2 - a1)}[c]

    for i, (cx, cy) in enumerate(velocities(2)):
        fi = rho * psi1(cx, u[0]) * psi1(cy, u[1])
        expect = e * fi + rho * (chi(cx, u[0]) * psi1(cy, u[1]) + psi1(cx, u[0]) * chi(cy, u[1]))
        np.testing.assert_allclose(g[i], expect, rtol=1e-12, atol=1e-15)


def test_geq_closed_form_d3q27_matches_operator_application():
    # the same derivation in 3D: the operators act on E = e + sum_a u_a^2/2 one axis at a time,
    # g_i = e f_i + rho [chi_x psi_y psi_z + psi_x chi_y psi_z + psi_x psi_y chi_z]
    rho, u, theta = _random_state(3, (5,), seed=18)
    e = np.random.default_rng(19).uniform(0.5, 2.0, size=rho.shape)
    g = eq.geq(rho, u, theta, e)

    def psi1(c, v):
        return {0: 1 - theta - v * v, 1: 0.5 * (theta + v * v + v), -1: 0.5 * (theta + v * v - v)}[c]

    def chi(c, v):
        a0 = 0.5 * v * v
        a1 = theta * v + 0.5 * v ** 3
        a2 = theta ** 2 + 2.5 * theta * v * v + 0.5 * v ** 4
        return {0: a0 - a2, 1: 0.5 * (a2 + a1), -1: 0.5 * (a2 - a1)}[c]

    for i, (cx, cy, cz) in enumerate(velocities(3)):
        px, py, pz = psi1(cx, u[0]), psi1(cy, u[1]), psi1(cz, u[2])
        expect = e * rho * px * py * pz + rho * (chi(cx, u[0]) * py * pz + px * chi(cy, u[1]) * pz
                                                 + px * py * chi(cz, u[2]))
        np.testing.assert_allclose(g[i], expect, rtol=1e-12, atol=1e-15)


def test_moments_inverts_equilibrium():
    rho, u, theta = _random_state(3, (3, 2, 2), seed=10)
    r, v = eq.moments(eq.feq(rho, u, theta))
    np.testing.assert_allclose(r, rho, rtol=1e-14)
    np.testing.assert_allclose(v, u, rtol=1e-12, atol=1e-15)
