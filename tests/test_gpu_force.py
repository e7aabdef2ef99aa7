"""GPU parity of the isothermal kernels with a uniform body force (Sec. II C: rho u =
sum c f + F/2, shifted equilibrium f^* at u + F/rho) against the FP64 CPU oracle.

Bars: float64 storage 1e-13 absolute on rho and u and on the stored post-collision
populations (indexing is exact, only rounding order differs); float32 storage rel-L2 <= 1e-5
on velocity. Analytic checks: exact acceleration of a uniform state, total momentum growth
by F per node and step, and the parabolic Poiseuille profile of Sec. III A.
"""
import functools

import numpy as np
import pytest

from gpu_util import announce, rel_l2, require_gpu
from oracle import bgk
from oracle.equilibrium import moments

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _lattice(*a, **k):
    from paper_2609_28679_amd.binding import Lattice
    return Lattice(*a, **k)


def _random_state(shape, D, seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.02 * rng.standard_normal(shape)
    u = 0.03 * rng.standard_normal((D,) + shape)
    return rho, u


CASES = [
    ("D2Q9", (29, 37), (2e-4, -1e-4)),
    ("D3Q27", (9, 11, 13), (1e-4, 2e-4, -3e-4)),
]


@pytest.mark.parametrize("streaming,steps", [("two", 7), ("one", 7), ("one", 8)])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("lattice,shape,F", CASES)
def test_forced_fp64_matches_oracle(lattice, shape, F, walls, streaming, steps):
    announce("%s %s force %s walls=%s fp64 %s buffer(s) %d steps"
             % (lattice, shape, F, walls, streaming, steps))
    D = len(shape)
    rho, u = _random_state(shape, D, seed=len(shape) * 10 + steps)
    tau = 0.7
    lat = _lattice(rho, u, lattice=lattice, storage="fp64", wall_y=walls, tau=tau,
                   streaming=streaming, force=F)
    lat.step(steps)
    rg, ug, _, tot = lat.moments()
    fg, _ = lat.populations()
    lat.close()
    Fv = np.asarray(F)
    om = bgk.omega_from_tau_lb(tau)
    f = bgk.run(bgk.init_equilibrium(rho, u), om, steps, walls, F=Fv)
    ro, uo = moments(f, F=Fv)
    assert np.abs(rg - ro).max() <= 1e-13
    assert np.abs(ug - uo).max() <= 1e-13
    # the stored state is the post-collision state of the same time
    assert np.abs(fg - bgk.collide(f, om, Fv)).max() <= 1e-13
    assert abs(tot[0] - ro.sum()) <= 1e-10
    for a in range(D):
        assert abs(tot[1 + a] - (ro * uo[a]).sum()) <= 1e-10


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("lattice,shape,F,steps", [
    ("D2Q9", (67, 130), (1e-5, -2e-5), 200),
    ("D3Q27", (20, 24, 33), (-1e-5, 1e-5, 2e-5), 60),
])
def test_forced_fp32_matches_oracle(lattice, shape, F, steps, walls):
    announce("%s %s force %s walls=%s fp32 %d steps" % (lattice, shape, F, walls, steps))
    D = len(shape)
    rho, u = _random_state(shape, D, seed=77)
    lat = _lattice(rho, u, lattice=lattice, storage="fp32", wall_y=walls, tau=0.6, force=F)
    lat.step(steps)
    _, ug, _, _ = lat.moments()
    lat.close()
    Fv = np.asarray(F)
    f = bgk.run(bgk.init_equilibrium(rho, u), bgk.omega_from_tau_lb(0.6), steps, walls, F=Fv)
    _, uo = moments(f, F=Fv)
    assert rel_l2(ug, uo) <= 1e-5


@pytest.mark.parametrize("streaming", ["two", "one"])
@pytest.mark.parametrize("lattice,shape,u0,F", [
    ("D2Q9", (6, 70), (0.01, -0.02), (1e-4, 3e-5)),
    ("D3Q27", (5, 6, 7), (0.01, -0.02, 0.005), (1e-4, 3e-5, -2e-5)),
])
def test_uniform_state_accelerates_exactly(lattice, shape, u0, F, streaming):
    # no gradients: every node gains F/rho of velocity per step, from the half-step value
    # u0 + F/(2 rho) of the equilibrium initialisation
    announce("%s uniform acceleration %s buffer(s)" % (lattice, streaming))
    D = len(shape)
    rho0 = 1.1
    rho = np.full(shape, rho0)
    u = np.asarray(u0).reshape((D,) + (1,) * D) * np.ones((D,) + shape)
    lat = _lattice(rho, u, lattice=lattice, storage="fp64", tau=0.7, streaming=streaming, force=F)
    for t in range(5):
        r, v, _, _ = lat.moments()
        expect = np.asarray(u0) + np.asarray(F) / (2 * rho0) + t * np.asarray(F) / rho0
        assert np.abs(v - expect.reshape((D,) + (1,) * D)).max() <= 1e-15
        assert np.abs(r - rho0).max() <= 1e-14
        lat.step(1)
    lat.close()


@pytest.mark.parametrize("lattice,shape,F", CASES)
def test_total_momentum_grows_by_the_force(lattice, shape, F):
    announce("%s momentum growth with diagnostics" % lattice)
    D = len(shape)
    rho, u = _random_state(shape, D, seed=3)
    lat = _lattice(rho, u, lattice=lattice, storage="fp64", tau=0.6, diag_every=1, force=F)
    lat.step(6)
    h = lat.diag_history()
    lat.close()
    assert h.shape[0] == 6
    nodes = rho.size
    growth = np.diff(h[:, 2:2 + D], axis=0)
    np.testing.assert_allclose(growth, np.tile(nodes * np.asarray(F), (5, 1)), rtol=1e-9)
    np.testing.assert_allclose(h[:, 1], rho.sum(), rtol=1e-13)


@functools.lru_cache(maxsize=None)
def _oracle_channel(ny, tau, F, steps):
    """The oracle's channel flow on a 3-wide lattice (the flow is uniform in x), started from
    the parabola, after `steps` steps: u_x(y)."""
    nu = (tau - 0.5) / 3.0
    y = np.arange(ny)
    u = np.zeros((2, ny, 3))
    u[0] = (F / (2 * nu) * (y + 0.5) * (ny - 0.5 - y))[:, None]
    Fv = np.array([F, 0.0])
    f = bgk.run(bgk.init_equilibrium(np.ones((ny, 3)), u), bgk.omega_from_tau_lb(tau), steps,
                walls_y=True, F=Fv)
    return moments(f, F=Fv)[1][0, :, 0]


@pytest.mark.parametrize("storage,tol", [("fp64", 1e-9), ("fp32", 1e-5)])
def test_poiseuille_profile(storage, tol):
    # Sec. III A: force-driven channel flow between half-way bounce-back walls at y = -1/2 and
    # y = ny - 1/2; steady profile u(y) = F/(2 rho nu) (y + 1/2)(ny - 1/2 - y). At tau = 1 the
    # scheme's steady state differs from the parabola only by the second-order error that the
    # oracle pins (below 3e-3 at ny = 24); the GPU profile is compared with the oracle's.
    ny, nx, tau, F = 24, 64, 1.0, 1e-6
    announce("D2Q9 Poiseuille ny=%d %s" % (ny, storage))
    nu = (tau - 0.5) / 3.0
    y = np.arange(ny)
    exact = F / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    rho = np.ones((ny, nx))
    u = np.zeros((2, ny, nx))
    u[0] = exact[:, None]
    lat = _lattice(rho, u, storage=storage, wall_y=True, tau=tau, force=(F, 0.0))
    lat.step(6000)
    _, ug, _, _ = lat.moments()
    lat.close()
    uo = _oracle_channel(ny, tau, F, 6000)
    assert rel_l2(ug[0], np.broadcast_to(uo[:, None], (ny, nx))) <= tol
    assert np.abs(ug[1]).max() <= 1e-6 * exact.max()
    assert rel_l2(uo, exact) <= 3e-3


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_womersley_time_varying_force(storage):
    # Sec. III A: pulsatile channel flow at Wo = 4 with the force changed before every step;
    # the GPU samples of the last period match the oracle's, and both the analytic solution
    from womersley import Case, oracle_samples
    case = Case(32)
    nx = 64
    announce("D2Q9 Womersley ny=%d %s %d steps" % (case.ny, storage, case.nsteps))
    rho = np.ones((case.ny, nx))
    u = np.zeros((2, case.ny, nx))
    u[0] = case.initial_ux()[:, None]
    lat = _lattice(rho, u, storage=storage, wall_y=True, tau=case.tau,
                   force=(case.force(0), 0.0))
    want = set(case.samples)
    gpu = {}
    for t in range(case.nsteps + 1):
        if t in want:
            _, ug, _, _ = lat.moments()
            assert np.abs(ug[0] - ug[0][:, :1]).max() <= 1e-6 * np.abs(ug[0]).max()
            gpu[t] = ug[0][:, 0].copy()
        lat.set_force((case.force(t + 1), 0.0))
        lat.step(1)
    lat.close()
    ref = oracle_samples(case)
    if storage == "fp64":  # rounding order only: the float64 bar on velocity
        assert max(np.abs(gpu[t] - ref[t]).max() for t in case.samples) <= 1e-13
    else:
        num = sum(((gpu[t] - ref[t]) ** 2).sum() for t in case.samples)
        den = sum((ref[t] ** 2).sum() for t in case.samples)
        assert np.sqrt(num / den) <= 1e-5
    assert case.rel_l2(gpu) <= 1.5e-3

