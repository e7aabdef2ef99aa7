"""GPU parity of the D3Q27 double-distribution kernels (two launches per step: fluxes, then the
collision) against the FP64 oracle.

Bars: float64 storage 1e-13 absolute on rho, u and T and on the stored post-collision
populations (exact indexing, rounding order only); float32 storage rel-L2 <= 1e-5 on velocity
and on temperature deviations. The oracle's D3Q27 double distribution applies the operator
definition of g^eq literally and is slow, so the lattices here are small but span several
workgroups in x and ragged tile edges.
"""
import numpy as np
import pytest

from gpu_util import announce, rel_l2, require_gpu
from oracle import ddf

pytestmark = pytest.mark.gpu

R, CV, P0 = 1.0 / 3.0, 5.0 / 6.0, 1.0 / 3.0
STENCIL = {0: "central", 1: "central", 2: "upwind"}


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _fields(shape, seed):
    rng = np.random.default_rng(seed)
    T = 0.9 + 0.05 * rng.standard_normal(shape)
    rho = P0 / (R * T) * (1 + 0.01 * rng.standard_normal(shape))
    u = 0.03 * rng.standard_normal((3,) + shape)  # no exact zeros (upwind side choice)
    return rho, u, T


def _run(rho, u, T, steps, storage, tau=0.7, **kw):
    from paper_2609_28679_amd.binding import Lattice
    lat = Lattice(rho, u, T, lattice="D3Q27", model="ddf", R=R, cv=CV, tau=tau,
                  storage=storage, **kw)
    lat.step(steps)
    r, v, t, tot = lat.moments()
    f, g = lat.populations()
    lat.close()
    return r, v, t, tot, f, g


# 0: plain; 1: sources and transport terms (the two launches); 2: sources only (with central
# Phi the one-launch step, which drops the transport terms at compile time)
EXTRA = [dict(), dict(force=(1e-4, -2e-4, 1e-4), heat_source=1e-4, prandtl=0.71,
                      eta_over_mu=1.5),
         dict(force=(1e-4, -2e-4, 1e-4), heat_source=1e-4)]


@pytest.mark.parametrize("extra", [0, 1, 2])
@pytest.mark.parametrize("phi", [1, 2, 0])
@pytest.mark.parametrize("walls", [True, False])
def test_fp64_matches_oracle(walls, phi, extra):
    kw = EXTRA[extra]
    shape = (5, 7, 9)
    announce("D3Q27 DDF fp64 %s walls=%s phi=%d extra=%s 5 steps" % (shape, walls, phi, kw))
    rho, u, T = _fields(shape, seed=31 + extra)
    steps, tau = 5, 0.7
    rg, ug, tg, tot, fg, gg = _run(rho, u, T, steps, "fp64", tau=tau, wall_y=walls, phi=phi,
                                   **kw)
    eta = kw.get("eta_over_mu")
    gas = ddf.Gas(R, CV, (tau - 0.5) * P0, prandtl=kw.get("prandtl", 1.0), eta_over_mu=eta)
    F = np.asarray(kw["force"]) if "force" in kw else None
    Q = kw.get("heat_source", 0.0)
    f, g = ddf.init_equilibrium(rho, u, T, gas)
    f, g = ddf.run(f, g, gas, steps, walls_y=walls, phi_on=phi > 0, stencil=STENCIL[phi],
                   F=F, Q=Q)
    ro, uo, to = ddf.temperature(f, g, gas, F=F, Q=Q)
    assert np.abs(rg - ro).max() <= 1e-13
    assert np.abs(ug - uo).max() <= 1e-13
    assert np.abs(tg - to).max() <= 1e-13
    ft, gt = ddf.collide(f, g, gas, walls, phi > 0, STENCIL[phi], F=F, Q=Q)
    assert np.abs(fg - ft).max() <= 1e-13
    assert np.abs(gg - gt).max() <= 1e-13
    assert abs(tot[0] - ro.sum()) <= 1e-10


def test_fp64_several_workgroups_in_x():
    shape = (3, 4, 300)
    announce("D3Q27 DDF fp64 %s walls phi=1 3 steps" % (shape,))
    rho, u, T = _fields(shape, seed=40)
    rg, ug, tg, _, _, _ = _run(rho, u, T, 3, "fp64", wall_y=True, phi=1)
    gas = ddf.Gas(R, CV, 0.2 * P0)
    f, g = ddf.run(*ddf.init_equilibrium(rho, u, T, gas), gas, 3, walls_y=True)
    ro, uo, to = ddf.temperature(f, g, gas)
    assert np.abs(ug - uo).max() <= 1e-13
    assert np.abs(tg - to).max() <= 1e-13


def test_fp32_matches_oracle():
    shape = (10, 8, 40)
    announce("D3Q27 DDF fp32 %s walls phi=1 20 steps" % (shape,))
    rho, u, T = _fields(shape, seed=41)
    _, ug, tg, _, _, _ = _run(rho, u, T, 20, "fp32", tau=0.6, wall_y=True, phi=1)
    gas = ddf.Gas(R, CV, 0.1 * P0)
    f, g = ddf.run(*ddf.init_equilibrium(rho, u, T, gas), gas, 20, walls_y=True)
    _, uo, to = ddf.temperature(f, g, gas)
    assert rel_l2(ug, uo) <= 1e-5
    assert rel_l2(tg - 0.9, to - 0.9) <= 1e-5


def test_conservation_with_diagnostics():
    shape = (16, 16, 64)
    announce("D3Q27 DDF fp64 %s periodic conservation 50 steps" % (shape,))
    rho, u, T = _fields(shape, seed=42)
    from paper_2609_28679_amd.binding import Lattice
    lat = Lattice(rho, u, T, lattice="D3Q27", model="ddf", R=R, cv=CV, tau=0.6,
                  storage="fp64", wall_y=False, phi=1, diag_every=10)
    m0 = lat.moments()[3]
    lat.step(50)
    h = lat.diag_history()
    lat.close()
    assert len(h) == 5
    assert np.all(np.abs(h[:, 1] - m0[0]) <= 1e-12 * m0[0])              # mass
    assert np.all(np.abs(h[:, 2:5] - m0[1:4]) <= 1e-12 * m0[0])           # momentum
    assert np.all(np.abs(h[:, 5] - m0[4]) <= 1e-12 * m0[4])               # total energy


@pytest.mark.parametrize("phi", [1, 0])
@pytest.mark.parametrize("walls", [True, False])
def test_fp32_ragged_lattice(walls, phi):
    # float32 storage on a 37 x 33 x 20 lattice (ragged workgroups in x, rows over several
    # workgroups), 4 steps: stored populations and velocity against the oracle
    shape = (20, 33, 37)
    announce("D3Q27 DDF fp32 %s walls=%s phi=%d 4 steps" % (shape, walls, phi))
    rho, u, T = _fields(shape, seed=43 + phi)
    tau = 0.7
    _, ug, tg, _, fg, gg = _run(rho, u, T, 4, "fp32", tau=tau, wall_y=walls, phi=phi)
    gas = ddf.Gas(R, CV, (tau - 0.5) * P0)
    f, g = ddf.run(*ddf.init_equilibrium(rho, u, T, gas), gas, 4, walls_y=walls, phi_on=phi > 0)
    ft, gt = ddf.collide(f, g, gas, walls, phi > 0, "central")
    assert np.abs(fg - ft).max() <= 2e-6 * np.abs(ft).max()
    assert np.abs(gg - gt).max() <= 2e-6 * np.abs(gt).max()
    _, uo, to = ddf.temperature(f, g, gas)
    assert rel_l2(ug, uo) <= 1e-5


@pytest.mark.parametrize("walls", [True, False])
def test_fp32_ragged_lattice_transport_control(walls):
    # the same ragged lattice with Pr 0.71 and bulk viscosity (T and u exchanged between tiles
    # like the fluxes in the one-launch step), 4 steps against the oracle
    shape = (20, 33, 37)
    announce("D3Q27 DDF fp32 %s walls=%s Pr 0.71 eta/mu 1.5 4 steps" % (shape, walls))
    rho, u, T = _fields(shape, seed=47)
    tau = 0.7
    _, ug, tg, _, fg, gg = _run(rho, u, T, 4, "fp32", tau=tau, wall_y=walls, phi=1,
                                prandtl=0.71, eta_over_mu=1.5)
    gas = ddf.Gas(R, CV, (tau - 0.5) * P0, prandtl=0.71, eta_over_mu=1.5)
    f, g = ddf.run(*ddf.init_equilibrium(rho, u, T, gas), gas, 4, walls_y=walls)
    ft, gt = ddf.collide(f, g, gas, walls, True, "central")
    assert np.abs(fg - ft).max() <= 2e-6 * np.abs(ft).max()
    assert np.abs(gg - gt).max() <= 2e-6 * np.abs(gt).max()
    _, uo, to = ddf.temperature(f, g, gas)
    assert rel_l2(ug, uo) <= 1e-5
    assert rel_l2(tg - tg.mean(), to - to.mean()) <= 1e-4


@pytest.mark.parametrize("walls", [True, False])
def test_fp64_tall_lattice_more_rows_than_grid_limit(walls):
    # a 7 x 3 x 2 state tiled 6300 times along z: 132300 (y, z) rows exceed two rows per
    # workgroup within the launch limit of 65535 workgroups, so each workgroup takes three. On a
    # z-periodic lattice the tiled state evolves as the small lattice's solution, tiled.
    reps = 6300
    small = (7, 3, 2)
    announce("D3Q27 DDF fp64 tall %s x %d along z, walls=%s, 3 steps" % (small, reps, walls))
    rho, u, T = _fields(small, seed=44)
    tile = lambda a: np.tile(a, (reps,) + (1,) * (a.ndim - 1))
    rg, ug, tg, _, _, _ = _run(tile(rho), np.stack([tile(c) for c in u]), tile(T), 3, "fp64",
                               wall_y=walls, phi=1)
    gas = ddf.Gas(R, CV, 0.2 * P0)
    f, g = ddf.run(*ddf.init_equilibrium(rho, u, T, gas), gas, 3, walls_y=walls)
    ro, uo, to = ddf.temperature(f, g, gas)
    assert np.abs(rg - tile(ro)).max() <= 1e-13
    assert np.abs(ug - np.stack([tile(c) for c in uo])).max() <= 1e-13
    assert np.abs(tg - tile(to)).max() <= 1e-13


@pytest.mark.parametrize("shape,walls", [((1, 3, 1), True), ((1, 1, 1), False), ((2, 1, 3), False)])
def test_fp64_one_node_wide(shape, walls):
    # lattices one node wide along some axes: every neighbour along such an axis is the node
    # itself (periodic) or a wall
    announce("D3Q27 DDF fp64 %s walls=%s 4 steps" % (shape, walls))
    rho, u, T = _fields(shape, seed=45)
    rg, ug, tg, _, fg, gg = _run(rho, u, T, 4, "fp64", wall_y=walls, phi=1)
    gas = ddf.Gas(R, CV, 0.2 * P0)
    f, g = ddf.run(*ddf.init_equilibrium(rho, u, T, gas), gas, 4, walls_y=walls)
    ro, uo, to = ddf.temperature(f, g, gas)
    assert np.abs(rg - ro).max() <= 1e-13
    assert np.abs(ug - uo).max() <= 1e-13
    assert np.abs(tg - to).max() <= 1e-13
    ft, gt = ddf.collide(f, g, gas, walls, True, "central")
    assert np.abs(fg - ft).max() <= 1e-13
    assert np.abs(gg - gt).max() <= 1e-13
