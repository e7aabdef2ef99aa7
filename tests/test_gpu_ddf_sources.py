"""GPU parity of the double-distribution kernel with a uniform body force F and heat source Q
(Sec. II C: half-step moments rho u = sum c f + F/2, rho E = sum g + (u.F + Q)/2; shifted
u*, theta*, T*; g* = g^eq(rho, u*, T*, theta*)) against the FP64 oracle.

Bars: float64 storage 1e-13 absolute on rho, u and T and on the stored post-collision
populations; float32 storage rel-L2 <= 1e-5 on velocity and temperature deviations. Exact
properties: isochoric heating raises T by Q/(rho c_v) per step, a uniform force leaves T
unchanged.
"""
import numpy as np
import pytest

from gpu_util import announce, rel_l2, require_gpu
from oracle import bgk, ddf
from paper_2609_28679_amd import inputs

pytestmark = pytest.mark.gpu

R, CV, P0 = 1.0 / 3.0, 5.0 / 6.0, 1.0 / 3.0
STENCIL = {0: "central", 1: "central", 2: "upwind"}


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _gas(tau):
    return ddf.Gas(R, CV, (tau - 0.5) * P0)


def _lattice(rho, u, T, **kw):
    from paper_2609_28679_amd.binding import Lattice
    return Lattice(rho, u, T, model="ddf", R=R, cv=CV, **kw)


def _random_fields(ny, nx, seed):
    rng = np.random.default_rng(seed)
    T = 0.9 + 0.05 * rng.standard_normal((ny, nx))
    rho = P0 / (R * T) * (1 + 0.01 * rng.standard_normal((ny, nx)))
    u = 0.02 * rng.standard_normal((2, ny, nx))  # no exact zeros (upwind side choice)
    return rho, u, T


@pytest.mark.parametrize("phi", [1, 2, 0])
@pytest.mark.parametrize("walls", [True, False])
@pytest.mark.parametrize("F,Q", [((2e-4, -1e-4), 0.0), ((0.0, 0.0), 3e-4),
                                 ((-1e-4, 2e-4), -2e-4)])
def test_sources_fp64_match_oracle(F, Q, walls, phi):
    announce("DDF fp64 sources F=%s Q=%g walls=%s phi=%d 300x37 9 steps" % (F, Q, walls, phi))
    rho, u, T = _random_fields(37, 300, seed=11)
    tau, steps = 0.7, 9
    lat = _lattice(rho, u, T, tau=tau, wall_y=walls, phi=phi, storage="fp64", force=F,
                   heat_source=Q)
    lat.step(steps)
    rg, ug, tg, _ = lat.moments()
    fg, gg = lat.populations()
    lat.close()
    gas = _gas(tau)
    Fv = np.asarray(F)
    f, g = ddf.init_equilibrium(rho, u, T, gas)
    # the context stores the post-collision state: creation collides the equilibrium once
    f, g = ddf.run(f, g, gas, steps, walls_y=walls, phi_on=phi > 0, stencil=STENCIL[phi],
                   F=Fv, Q=Q)
    ro, uo, to = ddf.temperature(f, g, gas, F=Fv, Q=Q)
    assert np.abs(rg - ro).max() <= 1e-13
    assert np.abs(ug - uo).max() <= 1e-13
    assert np.abs(tg - to).max() <= 1e-13
    ft, gt = ddf.collide(f, g, gas, walls, phi > 0, STENCIL[phi], F=Fv, Q=Q)
    assert np.abs(fg - ft).max() <= 1e-13
    assert np.abs(gg - gt).max() <= 1e-13


def test_sources_fp32_shear_layer():
    announce("DDF fp32 shear layer 128x64 walls phi=1 300 steps with F and Q")
    rho, u, T = inputs.thermal_shear_layer(128, seed=0, ny=64)
    F, Q = np.array([2e-6, 0.0]), 1e-6
    lat = _lattice(rho, u, T, tau=0.6, wall_y=True, phi=1, storage="fp32", force=F,
                   heat_source=Q)
    lat.step(300)
    _, ug, tg, _ = lat.moments()
    lat.close()
    gas = _gas(0.6)
    f, g = ddf.init_equilibrium(rho, u, T, gas)
    f, g = ddf.run(f, g, gas, 300, walls_y=True, F=F, Q=Q)
    _, uo, to = ddf.temperature(f, g, gas, F=F, Q=Q)
    assert rel_l2(ug, uo) <= 1e-5
    assert rel_l2(tg - 0.9, to - 0.9) <= 1e-5


@pytest.mark.parametrize("storage,tol", [("fp64", 2e-14), ("fp32", 1e-6)])
def test_isochoric_heating(storage, tol):
    # Sec. III B: a uniform heat source on a periodic box at rest raises T by exactly
    # Q / (rho c_v) per step (half a step already in the read-out at t = 0)
    announce("DDF isochoric heating %s" % storage)
    rho0, T0, Q = 1.2, 0.9, 1e-4
    shape = (8, 70)
    lat = _lattice(np.full(shape, rho0), np.zeros((2,) + shape), np.full(shape, T0), tau=0.6,
                   wall_y=False, phi=1, storage=storage, heat_source=Q)
    for t in range(6):
        r, v, T, _ = lat.moments()
        expect = T0 + Q / (2 * rho0 * CV) + t * Q / (rho0 * CV)
        assert np.abs(T - expect).max() <= tol * T0
        assert np.abs(v).max() <= tol
        lat.step(1)
    lat.close()


def test_uniform_force_keeps_temperature():
    announce("DDF uniform force fp64")
    rho0, T0 = 1.2, 0.9
    u0, F = np.array([0.02, 0.01]), np.array([1e-4, -2e-4])
    shape = (6, 40)
    lat = _lattice(np.full(shape, rho0), u0[:, None, None] * np.ones((2,) + shape),
                   np.full(shape, T0), tau=0.7, wall_y=False, phi=1, storage="fp64", force=F)
    T_first = None
    for t in range(6):
        _, v, T, _ = lat.moments()
        expect = u0 + F / (2 * rho0) + t * F / rho0
        assert np.abs(v - expect[:, None, None]).max() <= 1e-15
        T_first = T if T_first is None else T_first
        assert np.abs(T - T_first).max() <= 2e-14
        lat.step(1)
    lat.close()


def test_sources_changed_between_steps():
    # the context's collision at time t uses the sources set before the step that reached t
    # (creation: t = 0); the read-out uses those of the collision that produced the state
    announce("DDF fp64 sources switched between steps")
    rho, u, T = _random_fields(20, 33, seed=5)
    gas = _gas(0.6)
    plan = [((1e-4, 0.0), 2e-4, 3), ((0.0, -2e-4), 0.0, 2), ((0.0, 0.0), -1e-4, 2)]
    lat = _lattice(rho, u, T, tau=0.6, wall_y=True, phi=1, storage="fp64",
                   force=plan[0][0], heat_source=plan[0][1])
    # sources of the collision at each time t
    sched = [plan[0]]
    for F, Q, n in plan:
        sched += [(F, Q, 0)] * n
    f, g = ddf.init_equilibrium(rho, u, T, gas)
    t = 0
    for k, (F, Q, n) in enumerate(plan):
        if k:
            lat.set_force(F)
            lat.set_heat_source(Q)
        lat.step(n)
        for _ in range(n):
            Fp, Qp, _ = sched[t]
            ft, gt = ddf.collide(f, g, gas, True, True, "central", F=np.asarray(Fp), Q=Qp)
            f, g = bgk.stream(ft, True), bgk.stream(gt, True)
            t += 1
        _, ug, tg, _ = lat.moments()
        _, uo, to = ddf.temperature(f, g, gas, F=np.asarray(F), Q=Q)
        assert np.abs(ug - uo).max() <= 1e-13, k
        assert np.abs(tg - to).max() <= 1e-13, k
    lat.close()


@pytest.mark.parametrize("phi", [1, 2])
@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q27"])
def test_diagnostics_across_source_switches(lattice, phi):
    # a force and heat source change momentum and energy but conserve mass exactly; switching
    # them on and off between steps moves the step between launch shapes (D2Q9: taller rows on
    # the extended path; D3Q27: the one-launch step with and without sources, or with upwind
    # Phi the two sweeps on one row per workgroup, twice the plan's records), which write
    # different numbers of diagnostics records. The history's mass is the oracle's at every
    # recorded step only if each step's records alone are summed.
    announce("DDF fp64 %s phi=%d diagnostics with sources switched on and off" % (lattice, phi))
    if lattice == "D2Q9":
        rho, u, T = _random_fields(37, 70, seed=8)
        shape = (37, 70)
    else:
        rng = np.random.default_rng(9)
        shape = (6, 11, 70)
        T = 0.9 + 0.05 * rng.standard_normal(shape)
        rho = P0 / (R * T) * (1 + 0.01 * rng.standard_normal(shape))
        u = 0.02 * rng.standard_normal((3,) + shape)
    zero = (0.0,) * (2 if lattice == "D2Q9" else 3)
    on = (1e-4, -2e-4) if lattice == "D2Q9" else (1e-4, -2e-4, 5e-5)
    lat = _lattice(rho, u, T, lattice=lattice, tau=0.7, wall_y=False, phi=phi, storage="fp64",
                   diag_every=2)
    m0 = lat.moments()[3][0]
    for F, Q in [(zero, 0.0), (on, 2e-4), (zero, 0.0), (on, -1e-4)]:
        lat.set_force(F)
        lat.set_heat_source(Q)
        lat.step(4)
    h = lat.diag_history()
    lat.close()
    assert len(h) == 8
    assert np.all(np.abs(h[:, 1] - m0) <= 1e-12 * m0)


# ---- transport control: Prandtl number (q^c in g*) and bulk viscosity (alpha in theta*) ------

@pytest.mark.parametrize("phi", [1, 2])
@pytest.mark.parametrize("walls", [True, False])
@pytest.mark.parametrize("prandtl,eta,F,Q", [(0.5, -1.0, (0.0, 0.0), 0.0),
                                             (2.0, 2.0, (0.0, 0.0), 0.0),
                                             (1.0, 0.0, (1e-4, -2e-4), 1e-4),
                                             (0.71, 1.5, (-1e-4, 1e-4), -2e-4)])
def test_transport_control_fp64_matches_oracle(prandtl, eta, F, Q, walls, phi):
    announce("DDF fp64 Pr=%g eta/mu=%g F=%s Q=%g walls=%s phi=%d 300x37 9 steps"
             % (prandtl, eta, F, Q, walls, phi))
    rho, u, T = _random_fields(37, 300, seed=21)
    tau, steps = 0.7, 9
    lat = _lattice(rho, u, T, tau=tau, wall_y=walls, phi=phi, storage="fp64", force=F,
                   heat_source=Q, prandtl=prandtl, eta_over_mu=eta)
    lat.step(steps)
    rg, ug, tg, _ = lat.moments()
    fg, gg = lat.populations()
    lat.close()
    gas = ddf.Gas(R, CV, (tau - 0.5) * P0, prandtl=prandtl,
                  eta_over_mu=None if eta < 0 else eta)
    Fv = np.asarray(F)
    f, g = ddf.init_equilibrium(rho, u, T, gas)
    f, g = ddf.run(f, g, gas, steps, walls_y=walls, stencil=STENCIL[phi], F=Fv, Q=Q)
    ro, uo, to = ddf.temperature(f, g, gas, F=Fv, Q=Q)
    assert np.abs(rg - ro).max() <= 1e-13
    assert np.abs(ug - uo).max() <= 1e-13
    assert np.abs(tg - to).max() <= 1e-13
    ft, gt = ddf.collide(f, g, gas, walls, True, STENCIL[phi], F=Fv, Q=Q)
    assert np.abs(fg - ft).max() <= 1e-13
    assert np.abs(gg - gt).max() <= 1e-13


def test_transport_control_fp32_shear_layer():
    announce("DDF fp32 shear layer 128x64 walls Pr 0.71 eta/mu 1 300 steps")
    rho, u, T = inputs.thermal_shear_layer(128, seed=0, ny=64)
    lat = _lattice(rho, u, T, tau=0.6, wall_y=True, phi=1, storage="fp32", prandtl=0.71,
                   eta_over_mu=1.0)
    lat.step(300)
    _, ug, tg, _ = lat.moments()
    lat.close()
    gas = ddf.Gas(R, CV, 0.1 * P0, prandtl=0.71, eta_over_mu=1.0)
    f, g = ddf.init_equilibrium(rho, u, T, gas)
    f, g = ddf.run(f, g, gas, 300, walls_y=True)
    _, uo, to = ddf.temperature(f, g, gas)
    assert rel_l2(ug, uo) <= 1e-5
    assert rel_l2(tg - 0.9, to - 0.9) <= 1e-5
