"""Full-size checks in the launch configurations that bench.py times, for the workloads with a
body force, heat source, transport control, a van der Waals fluid (D2Q9 and D3Q27),
non-equilibrium extrapolation walls and the D3Q27 double distribution: the GPU state after one
or two steps from the seeded initial fields against the oracle run from the same fields, element
by element on whole lattices, row slabs or node neighbourhoods that the oracle can compute
(windows of the initial fields wide enough that the checked nodes are exact, tests/windows.py).

The double-distribution context stores the post-collision state of t = 0 (its creation collides
the initial equilibrium once); after one step it holds the post-collision state of t = 1, which
is the oracle's collide(run(init, 1))."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from oracle import bgk, ddf
from paper_2609_28679_amd import inputs
from windows import periodic_box, rows, wall_blocks

pytestmark = pytest.mark.gpu

R, CV, P0 = 1.0 / 3.0, 5.0 / 6.0, 1.0 / 3.0
MARGIN = 6  # rows beyond a checked row: one step reaches 3 (collide, pull, collide)


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _lattice(*a, **k):
    from paper_2609_28679_amd.binding import Lattice
    return Lattice(*a, **k)


def _close(got, want, tol=2e-6):
    return np.abs(got - want).max() <= tol * np.abs(want).max()


def _gpu_state(lat, steps):
    lat.step(steps)
    out = lat.populations()
    lat.close()
    return out


def test_forced_d2q9_2048_one_buffer():
    announce("D2Q9 2048^2 fp32 one buffer, uniform force (bench configuration): 2 steps")
    rho, u = inputs.random_phase_turbulence_2d(2048, seed=0)
    F = np.array([1e-6, 0.0])
    f_next, _ = _gpu_state(_lattice(rho, u, tau=0.6, force=tuple(F)), 2)
    om = bgk.omega_from_tau_lb(0.6)
    want = bgk.collide(bgk.run(bgk.init_equilibrium(rho, u), om, 2, F=F), om, F)
    assert _close(f_next, want)


def test_forced_d3q27_256():
    announce("D3Q27 256^3 fp32, uniform force (bench configuration): 2 steps on 4 slabs")
    n, steps = 256, 2
    rho, u = inputs.taylor_green_3d(n, 0.05)
    F = np.array([1e-6, 0.0, 0.0])
    f_next, _ = _gpu_state(_lattice(rho, u, lattice="D3Q27", tau=0.55, force=tuple(F)), steps)
    om = bgk.omega_from_tau_lb(0.55)
    for z in (0, 1, 128, 255):
        iz = [(z + d) % n for d in range(-steps, steps + 1)]
        want = bgk.collide(bgk.run(bgk.init_equilibrium(rho[iz], u[:, iz]), om, steps, F=F),
                           om, F)[:, steps]
        assert _close(f_next[:, z], want), z


def _ddf_oracle_post(rho, u, T, gas, steps, F=None, Q=0.0, neq=None, walls_y=True):
    """Post-collision populations after `steps` steps from the initial fields (see module)."""
    f, g = ddf.init_equilibrium(rho, u, T, gas)
    f, g = ddf.run(f, g, gas, steps, walls_y=walls_y, F=F, Q=Q, neq=neq)
    return ddf.collide(f, g, gas, walls_y or neq is not None, True, "central", F=F, Q=Q,
                       neq=neq)


def _ddf_rows(fields, gpu, gas, check, F=None, Q=0.0):
    """D2Q9 double distribution with bounce-back walls at the lattice ends: the rows in `check`
    after one step, each from a slab of the initial fields MARGIN rows around it (a slab that
    reaches the lattice's end has the real wall there)."""
    rho, u, T = fields
    f_next, g_next = gpu
    n = rho.shape[0]
    for c in check:
        lo, hi = max(c - MARGIN, 0), min(c + MARGIN + 1, n)
        ft, gt = _ddf_oracle_post(rows(rho, lo, hi), rows(u, lo, hi), rows(T, lo, hi), gas, 1,
                                  F=F, Q=Q)
        assert _close(f_next[:, c], ft[:, c - lo]), c
        assert _close(g_next[:, c], gt[:, c - lo]), c


@pytest.mark.parametrize("case", ["sources", "transport"])
def test_ddf_4096_extended(case):
    n = 4096
    announce("DDF 4096^2 fp32 walls, %s (bench configuration): one step at sampled rows" % case)
    fields = inputs.thermal_shear_layer(n, seed=0)
    if case == "sources":
        kw, F, Q = dict(force=(1e-7, 0.0), heat_source=1e-8), np.array([1e-7, 0.0]), 1e-8
        gas = ddf.Gas(R, CV, 0.1 * P0)
    else:
        kw, F, Q = dict(prandtl=0.71, eta_over_mu=1.0), None, 0.0
        gas = ddf.Gas(R, CV, 0.1 * P0, prandtl=0.71, eta_over_mu=1.0)
    gpu = _gpu_state(_lattice(*fields, model="ddf", tau=0.6, wall_y=True, phi=1, **kw), 1)
    _ddf_rows(fields, gpu, gas, (0, 1, 2047, n - 2, n - 1), F, Q)


def test_ddf_4096_vdw():
    n = 4096
    announce("DDF 4096^2 fp32 walls, van der Waals fluid (bench configuration): one step at "
             "sampled rows")
    _, u, T = inputs.thermal_shear_layer(n, seed=0, T0=1.4, dT=0.03)
    rho = np.ones_like(T)
    gpu = _gpu_state(_lattice(rho, u, T, model="ddf", tau=0.6, wall_y=True, phi=1,
                              vdw=(0.27, 0.2)), 1)
    gas = ddf.Gas(R, CV, 0.1 * P0, a=0.27, b=0.2)
    _ddf_rows((rho, u, T), gpu, gas, (0, 1, 2047, n - 2, n - 1))


def test_ddf_4096_neq_walls():
    n = 4096
    announce("DDF 4096^2 fp32 non-equilibrium extrapolation walls (bench configuration): one step")
    rho, u, T = inputs.thermal_shear_layer(n, seed=0)
    f_next, g_next = _gpu_state(_lattice(rho, u, T, model="ddf", tau=0.6, phi=1,
                                         neq_walls=dict(u=((-0.05, 0.0), (0.05, 0.0)),
                                                        T=(0.8, 1.0))), 1)
    gas = ddf.Gas(R, CV, 0.1 * P0)
    walls = ddf.NeqWalls((-0.05, 0.0), 0.8, (0.05, 0.0), 1.0)
    # the first and last MARGIN + 2 rows stacked: both walls are real, the junction far away
    d = MARGIN + 2
    ft, gt = _ddf_oracle_post(wall_blocks(rho, d), wall_blocks(u, d), wall_blocks(T, d), gas, 1,
                              neq=walls, walls_y=False)
    for k, c in ((0, 0), (1, 1), (2 * d - 2, n - 2), (2 * d - 1, n - 1)):
        assert _close(f_next[:, c], ft[:, k]), c
        assert _close(g_next[:, c], gt[:, k]), c
    # an interior row is an ordinary row (bounce-back walls of the slab never reach it)
    lo, hi = 2047 - MARGIN, 2047 + MARGIN + 1
    ft, gt = _ddf_oracle_post(rows(rho, lo, hi), rows(u, lo, hi), rows(T, lo, hi), gas, 1)
    assert _close(f_next[:, 2047], ft[:, MARGIN])
    assert _close(g_next[:, 2047], gt[:, MARGIN])


def _ddf3_nodes(fields, gpu, gas, n, seed, F=None, Q=0.0):
    """Sampled nodes of a periodic D3Q27 double-distribution step, each from the periodic box of
    the initial fields of radius 4 around it (one step reaches 3)."""
    rho, u, T = fields
    f_next, g_next = gpu
    rng = np.random.default_rng(seed)
    nodes = [(0, 0, 0), (255, 128, 1), (17, 255, 254)] + [tuple(v) for v in rng.integers(0, n, (3, 3))]
    r = 4
    for z, y, x in nodes:
        c = (z, y, x)
        ft, gt = _ddf_oracle_post(periodic_box(rho, c, r), periodic_box(u, c, r, lead=1),
                                  periodic_box(T, c, r), gas, 1, F=F, Q=Q, walls_y=False)
        assert _close(f_next[:, z, y, x], ft[:, r, r, r]), c
        assert _close(g_next[:, z, y, x], gt[:, r, r, r]), c


@pytest.mark.parametrize("case", ["sources", "transport"])
def test_ddf3_256_extended(case):
    n = 256
    announce("D3Q27 DDF 256^3 fp32 periodic, %s (bench configuration): one step at sampled "
             "nodes" % case)
    fields = inputs.thermal_taylor_green_3d(n, 0.05)
    if case == "sources":
        kw, F, Q = dict(force=(1e-7, 0.0, 0.0), heat_source=1e-8), np.array([1e-7, 0.0, 0.0]), 1e-8
        gas = ddf.Gas(R, CV, 0.1 * P0)
    else:
        kw, F, Q = dict(prandtl=0.71, eta_over_mu=1.0), None, 0.0
        gas = ddf.Gas(R, CV, 0.1 * P0, prandtl=0.71, eta_over_mu=1.0)
    gpu = _gpu_state(_lattice(*fields, lattice="D3Q27", model="ddf", tau=0.6, phi=1, **kw), 1)
    _ddf3_nodes(fields, gpu, gas, n, seed=5, F=F, Q=Q)


def test_ddf3_256_vdw():
    n = 256
    announce("D3Q27 DDF 256^3 fp32 periodic, van der Waals fluid (bench configuration): one "
             "step at sampled nodes")
    _, u = inputs.taylor_green_3d(n, 0.05)
    rho, T = np.ones(u.shape[1:]), np.full(u.shape[1:], 1.4)
    gpu = _gpu_state(_lattice(rho, u, T, lattice="D3Q27", model="ddf", tau=0.6, phi=1,
                              vdw=(0.27, 0.2)), 1)
    _ddf3_nodes((rho, u, T), gpu, ddf.Gas(R, CV, 0.1 * P0, a=0.27, b=0.2), n, seed=4)


def test_ddf3_256_neq_walls():
    n = 256
    announce("D3Q27 DDF 256^3 fp32 NEQ walls (bench configuration): one step at sampled nodes "
             "next to and on the walls")
    rho, u, T = inputs.thermal_taylor_green_3d(n, 0.05)
    f_next, g_next = _gpu_state(_lattice(rho, u, T, lattice="D3Q27", model="ddf", tau=0.6, phi=1,
                                         neq_walls=dict(u=((-0.05, 0.0), (0.05, 0.0)),
                                                        T=(0.8, 1.0))), 1)
    gas = ddf.Gas(R, CV, 0.1 * P0)
    walls = ddf.NeqWalls((-0.05, 0.0, 0.0), 0.8, (0.05, 0.0, 0.0), 1.0)
    # columns of the first and last d planes in y, a periodic box of radius r in z and x
    d, r = 6, 4
    for z, x in ((0, 0), (131, 255), (7, 64)):
        iz = [(z + k) % n for k in range(-r, r + 1)]
        ix = [(x + k) % n for k in range(-r, r + 1)]

        def col(a, lead=0):
            b = a[(Ellipsis,) + np.ix_(iz, list(range(n)), ix)] if lead else a[np.ix_(iz, list(range(n)), ix)]
            return wall_blocks(b, d, axis=-2)

        ft, gt = _ddf_oracle_post(col(rho), col(u, 1), col(T), gas, 1, neq=walls, walls_y=False)
        for k, y in ((0, 0), (1, 1), (2 * d - 2, n - 2), (2 * d - 1, n - 1)):
            assert _close(f_next[:, z, y, x], ft[:, r, k, r]), (z, y, x)
            assert _close(g_next[:, z, y, x], gt[:, r, k, r]), (z, y, x)


def test_ddf3_256():
    n = 256
    announce("D3Q27 DDF 256^3 fp32 periodic (bench configuration): one step at sampled nodes")
    fields = inputs.thermal_taylor_green_3d(n, 0.05)
    gpu = _gpu_state(_lattice(*fields, lattice="D3Q27", model="ddf", tau=0.6, phi=1), 1)
    _ddf3_nodes(fields, gpu, ddf.Gas(R, CV, 0.1 * P0), n, seed=3)
