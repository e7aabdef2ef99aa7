"""Womersley flow (Sec. III A): a channel between half-way bounce-back walls at y = -1/2 and
y = ny - 1/2 driven by the body force F_x(t) = F0 cos(Omega t). The analytic solution of
du/dt = nu d2u/dy2 + F_x(t)/rho with u = 0 on the walls is
    u(y, t) = Re{ F0 / (i Omega rho) [1 - cosh(l (y - yc)) / cosh(l ny / 2)] exp(i Omega t) },
l = sqrt(i Omega / nu), yc = (ny - 1)/2, and the Womersley number is Wo = (ny/2) sqrt(Omega/nu).
Test infrastructure shared by the oracle pin and the GPU test: the closed form, the case set-up
and the oracle's run of the case."""
import numpy as np

from oracle import bgk
from oracle.equilibrium import moments


def analytic(y, t, ny, omega_t, nu, F0, rho=1.0):
    lam = np.sqrt(1j * omega_t / nu)
    yc = (ny - 1) / 2.0
    U = F0 / (1j * omega_t * rho) * (1 - np.cosh(lam * (y - yc)) / np.cosh(lam * ny / 2.0))
    return (U * np.exp(1j * omega_t * t)).real


class Case:
    """Diffusive scaling: Omega = nu (2 Wo / ny)^2, F0 = 1e-5 (8 / ny)^2 (velocity amplitude
    independent of ny). `periods` periods are run; the last one is sampled at `phases` times."""

    def __init__(self, ny, Wo=4.0, tau=1.0, periods=5, phases=16):
        self.ny, self.tau = ny, tau
        self.nu = (tau - 0.5) / 3.0
        self.Om = self.nu * (2 * Wo / ny) ** 2
        self.F0 = 1e-5 * (8.0 / ny) ** 2
        T = 2 * np.pi / self.Om
        self.nsteps = int(round(periods * T))
        self.samples = sorted(set(int(round((periods - 1) * T + k * T / phases))
                                  for k in range(phases)))
        self.y = np.arange(ny)

    def force(self, t):
        return self.F0 * np.cos(self.Om * t)

    def exact(self, t):
        return analytic(self.y, t, self.ny, self.Om, self.nu, self.F0)

    def initial_ux(self):
        # the read-out adds F(0)/2 to the momentum, so the populations start from
        # u(y, 0) - F(0)/2 to read back the analytic u(y, 0)
        return self.exact(0) - self.force(0) / 2.0

    def rel_l2(self, ux_by_t):
        """ux_by_t: {t: u_x(y)} at the sample times."""
        num = sum(((ux_by_t[t] - self.exact(t)) ** 2).sum() for t in self.samples)
        den = sum((self.exact(t) ** 2).sum() for t in self.samples)
        return float(np.sqrt(num / den))


def oracle_samples(case):
    """The oracle's run of the case on a 3-wide channel (the flow is uniform in x): {t: u_x(y)}
    at the sample times, the force F(t) entering the collision and the read-out at time t."""
    u = np.zeros((2, case.ny, 3))
    u[0] = case.initial_ux()[:, None]
    f = bgk.init_equilibrium(np.ones((case.ny, 3)), u)
    om = bgk.omega_from_tau_lb(case.tau)
    out = {}
    want = set(case.samples)
    for t in range(case.nsteps + 1):
        Fv = np.array([case.force(t), 0.0])
        if t in want:
            out[t] = moments(f, F=Fv)[1][0, :, 0]
        f = bgk.stream(bgk.collide(f, om, Fv), walls_y=True)
    return out
