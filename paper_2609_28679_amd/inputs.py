"""Seeded synthetic initial fields (float64, host memory).

This module only builds input data: macroscopic initial fields, harvest plans and initial
network weights. It contains none of the lattice Boltzmann arithmetic and is the one piece
shared by the HIP path and the CPU reference. Random numbers come from
numpy.random.default_rng(seed) (PCG64).

Array conventions: node arrays are indexed [y, x] in 2D and [z, y, x] in 3D; velocity arrays
carry the component first, u[a] with a = x, y (, z).
"""
import numpy as np

RMS_MACH_TURB = 0.05
CS = 1.0 / np.sqrt(3.0)


def taylor_green_2d(nx, ny, u0, rho0=1.0):
    """2D Taylor-Green vortex on integer node coordinates, k = 2 pi / n per axis.

    u_x = -u0 cos(k x) sin(k y),  u_y = u0 sin(k x) cos(k y),  rho = rho0.
    """
    kx = 2.0 * np.pi / nx
    ky = 2.0 * np.pi / ny
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    u = np.empty((2, ny, nx))
    u[0] = -u0 * np.cos(kx * x) * np.sin(ky * y)
    u[1] = u0 * np.sin(kx * x) * np.cos(ky * y)
    rho = np.full((ny, nx), float(rho0))
    return rho, u


def taylor_green_3d(n, u0, rho0=1.0):
    """3D Taylor-Green vortex on an n^3 periodic box, k = 2 pi / n.

    u = u0 sin(kx) cos(ky) cos(kz),  v = -u0 cos(kx) sin(ky) cos(kz),  w = 0.
    """
    k = 2.0 * np.pi / n
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    u = np.empty((3, n, n, n))
    u[0] = u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    u[1] = -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    u[2] = 0.0
    rho = np.full((n, n, n), float(rho0))
    return rho, u


def thermal_taylor_green_3d(n, u0, T0=0.9, P0=1.0 / 3.0, R=1.0 / 3.0):
    """The 3D Taylor-Green velocity of taylor_green_3d at uniform temperature T0 and pressure
    P0 (ideal gas, rho = P0 / (R T0)): the double-distribution workload in 3D."""
    _, u = taylor_green_3d(n, u0)
    T = np.full((n, n, n), float(T0))
    rho = np.full((n, n, n), P0 / (R * T0))
    return rho, u, T


def random_phase_turbulence_2d(n, seed, kmax_frac=0.125, rms_mach=RMS_MACH_TURB):
    """Divergence-free random-phase velocity field with energy spectrum E(k) ~ k^(-5/3).

    Stream function amplitude |psi_hat| ~ |k|^(-7/3) on 1 <= |k| <= kmax_frac * n (integer
    wavenumbers), zero elsewhere; phases uniform on [0, 2 pi) drawn in np.fft index order;
    u = d psi/dy, v = -d psi/dx (spectral); scaled so that sqrt(<|u|^2>) = rms_mach * c_s.
    rho = 1.
    """
    rng = np.random.default_rng(seed)
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    ky, kx = np.meshgrid(k1, k1, indexing="ij")
    kmag = np.sqrt(kx * kx + ky * ky)
    amp = np.zeros((n, n))
    band = (kmag >= 1.0) & (kmag <= kmax_frac * n)
    amp[band] = kmag[band] ** (-7.0 / 3.0)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(n, n))
    psi = np.real(np.fft.ifft2(amp * np.exp(1j * phase)))
    psi_hat = np.fft.fft2(psi)
    two_pi_over_n = 2.0 * np.pi / n
    u = np.empty((2, n, n))
    u[0] = np.real(np.fft.ifft2(1j * ky * two_pi_over_n * psi_hat))
    u[1] = np.real(np.fft.ifft2(-1j * kx * two_pi_over_n * psi_hat))
    rms = np.sqrt(np.mean(u[0] ** 2 + u[1] ** 2))
    u *= rms_mach * CS / rms
    rho = np.ones((n, n))
    return rho, u


def thermal_shear_layer(n, seed, ny=None, ushear=0.05, dT=0.1, T0=0.9, P0=1.0 / 3.0,
                        R=1.0 / 3.0, pert=5e-4, modes=8):
    """Thermal shear layer between walls at y = -1/2 and y = ny - 1/2.

    s = (y - y_c)/delta with y_c = (ny - 1)/2 and delta = n/128 (at least 1);
    u_x = ushear tanh(s);  T = T0 + dT tanh(s);  uniform pressure P0, rho = P0 / (R T);
    the default T0 = 0.9 keeps T in [0.8, 1.0], i.e. theta = R T <= 1/3 with R = 1/3;
    u_y = pert * sum_{m=1..modes} a_m sin(2 pi m x / n + phi_m) exp(-s^2),
    with a_m and phi_m / (2 pi) uniform on [0, 1) from the seed.
    Returns rho, u (2, ny, n), T.
    """
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, size=modes)
    ph = 2.0 * np.pi * rng.uniform(0.0, 1.0, size=modes)
    delta = max(n / 128.0, 1.0)
    yc = 0.5 * (ny - 1)
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(n, dtype=np.float64),
                       indexing="ij")
    s = (y - yc) / delta
    u = np.empty((2, ny, n))
    u[0] = ushear * np.tanh(s)
    pert_x = np.zeros_like(x)
    for m in range(modes):
        pert_x += a[m] * np.sin(2.0 * np.pi * (m + 1) * x / n + ph[m])
    u[1] = pert * pert_x * np.exp(-s * s)
    T = T0 + dT * np.tanh(s)
    rho = P0 / (R * T)
    return rho, u, T


def harvest_plan(n_nodes, n_samples, steps, seed):
    """Random (step, node) pairs for training-data harvest: for every step in `steps`,
    n_samples // len(steps) distinct node indices in [0, n_nodes), sorted."""
    rng = np.random.default_rng(seed)
    per = n_samples // len(steps)
    plan = []
    for s in steps:
        idx = np.sort(rng.choice(n_nodes, size=per, replace=False)).astype(np.int64)
        plan.append((int(s), idx))
    return plan


def mlp_init(seed, n_in=12, n_hid=64, n_out=9):
    """Initial weights: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for W and b, float64.

    Returns [W1 (n_hid, n_in), b1, W2 (n_hid, n_hid), b2, W3 (n_out, n_hid), b3].
    """
    rng = np.random.default_rng(seed)
    out = []
    for fan_in, fan_out in ((n_in, n_hid), (n_hid, n_hid), (n_hid, n_out)):
        lim = 1.0 / np.sqrt(fan_in)
        out.append(rng.uniform(-lim, lim, size=(fan_out, fan_in)))
        out.append(rng.uniform(-lim, lim, size=fan_out))
    return out
