"""Pins of the surrogate reference: finite-difference gradients, the exact projection,
bfloat16 rounding against torch's conversion, GELU and the closed-form first Adam step."""
import numpy as np
import pytest
import torch

from oracle import mlp
from oracle.equilibrium import feq
from oracle.lattice import VARSIGMA2, velocities
from paper_2609_28679_amd import inputs


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.95, 1.05, n)
    u = rng.uniform(-0.05, 0.05, (2, n))
    f = feq(rho, u, VARSIGMA2).T + rng.normal(0.0, 2e-4, (n, 9))
    omega = rng.choice([1 / 0.51, 1 / 0.6, 1.0], n)
    return f, omega


def test_round_bf16_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        [0.0, -0.0, 1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 65504.0, 1e-40]])
    ours = mlp.round_bf16(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)
    # ties to even
    assert mlp.round_bf16(np.array([1 + 2 ** -8]))[0] == 1.0
    assert mlp.round_bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6


def test_gelu_limits_and_derivative():
    z = np.linspace(-6, 6, 101)
    assert mlp.gelu(np.array(0.0)) == 0.0
    np.testing.assert_allclose(mlp.gelu(np.array([10.0])), [10.0], rtol=1e-12)
    assert abs(mlp.gelu(np.array(-10.0))) < 1e-12
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)
    # the tanh form tracks the exact erf form to within about 1e-3
    from scipy.special import erf
    exact = 0.5 * z * (1 + erf(z / np.sqrt(2)))
    assert np.abs(mlp.gelu(z) - exact).max() < 1e-3


def test_projection_is_exact_and_idempotent():
    y = np.random.default_rng(1).standard_normal((50, 9))
    p = mlp.project(y)
    C = mlp.constraint_matrix()
    np.testing.assert_allclose(p @ C.T, 0.0, atol=1e-14)
    np.testing.assert_allclose(mlp.project(p), p, atol=1e-14)
    # components already in the subspace are untouched
    z = mlp.project(np.random.default_rng(2).standard_normal((5, 9)))
    np.testing.assert_allclose(mlp.project(z), z, atol=1e-14)


def test_targets_are_the_plain_collision_and_keep_invariants():
    f, omega = _batch(64, 3)
    t = mlp.targets(f, omega)
    C = mlp.constraint_matrix()
    np.testing.assert_allclose(t @ C.T, 0.0, atol=1e-9)
    # BGK: f~ - f^eq = (1 - omega)(f - f^eq)
    x, fe, rho = mlp.features(f, omega)
    np.testing.assert_allclose(t, (1 - omega)[:, None] * x[:, :9], rtol=1e-10, atol=1e-13)


def test_backward_matches_central_finite_differences():
    f, omega = _batch(16, 4)
    x, _, _ = mlp.features(f, omega)
    t = mlp.targets(f, omega)
    params = inputs.mlp_init(5)

    def L(ps):
        y, _ = mlp.forward(ps, x)
        return mlp.loss(y, t)

    y, cache = mlp.forward(params, x)
    grads = mlp.backward(params, cache, y, t)
    rng = np.random.default_rng(6)
    for k, p in enumerate(params):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in p.shape)
            h = 1e-6 * max(1.0, abs(p[idx]))
            pp = [q.copy() for q in params]
            pm = [q.copy() for q in params]
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (L(pp) - L(pm)) / (2 * h)
            assert grads[k][idx] == pytest.approx(fd, rel=1e-6, abs=1e-12)


def test_adam_first_step_closed_form():
    # t = 1: m_hat = g, v_hat = g^2, so the step is lr g / (|g| + eps)
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -1e-3, 0.0])]
    opt = mlp.Adam(lr=1e-3)
    (q,) = opt.step(p, g)
    np.testing.assert_allclose(q, p[0] - 1e-3 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-15)


def test_adam_constant_gradient_steps_closed_form():
    # A constant gradient g gives m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the
    # bias-corrected moments are g and g^2 at every t and each step moves a parameter by
    # exactly lr g / (|g| + eps). A wrong bias-correction power (or a missing correction)
    # breaks this from t = 2 on.
    lr, eps = 2e-3, 1e-8
    g = np.array([0.5, -1e-3, 3e-7, -40.0])
    p0 = np.array([1.0, -2.0, 3.0, 0.25])
    opt = mlp.Adam(lr=lr, eps=eps)
    p = [p0.copy()]
    step = lr * g / (np.abs(g) + eps)
    for t in range(1, 6):
        before = p[0].copy()
        p = opt.step(p, [g.copy()])
        np.testing.assert_allclose(before - p[0], step, rtol=1e-12, atol=0)
        np.testing.assert_allclose(p[0], p0 - t * step, rtol=1e-13)
    # the two moment estimates themselves
    np.testing.assert_allclose(opt.m[0], (1 - 0.9 ** 5) * g, rtol=1e-14)
    np.testing.assert_allclose(opt.v[0], (1 - 0.999 ** 5) * g * g, rtol=1e-12)


def test_adam_zero_gradient_after_one_step_decays_geometrically():
    # g_1 = g, then g_t = 0: m_t = b1^(t-1) (1 - b1) g and v_t = b2^(t-1) (1 - b2) g^2, so for
    # |g| >> eps the step at t is lr (b1 / sqrt(b2))^(t-1) sqrt(1 - b2^t) / (1 - b1^t)
    # * (1 - b1) / sqrt(1 - b2) * sign(g): a ratio of 0.9 / sqrt(0.999) between late steps.
    lr = 1e-3
    g = np.array([2.0, -3.0])
    opt = mlp.Adam(lr=lr, eps=0.0)
    p = [np.zeros(2)]
    steps = []
    for t in range(1, 8):
        before = p[0].copy()
        p = opt.step(p, [g if t == 1 else np.zeros(2)])
        steps.append(before - p[0])
    for t, d in enumerate(steps, start=1):
        exp = lr * (0.9 / np.sqrt(0.999)) ** (t - 1) * np.sqrt(1 - 0.999 ** t) / (1 - 0.9 ** t) \
            * 0.1 / np.sqrt(0.001) * np.sign(g)
        np.testing.assert_allclose(d, exp, rtol=1e-12)


def test_surrogate_with_zero_tolerance_is_the_plain_collision():
    f, omega = _batch(128, 7)
    params = inputs.mlp_init(8)
    out, fb = mlp.surrogate_collide(params, f, omega, tol=0.0)
    x, fe, rho = mlp.features(f, omega)
    plain = f + omega[:, None] * (fe - f)
    np.testing.assert_array_equal(out, plain)
    assert fb.all()


def test_surrogate_keeps_mass_and_momentum():
    f, omega = _batch(128, 9)
    out, _ = mlp.surrogate_collide(inputs.mlp_init(10), f, omega, tol=1e9)
    c = velocities(2).astype(np.float64)
    np.testing.assert_allclose(out.sum(axis=1), f.sum(axis=1), rtol=1e-13)
    np.testing.assert_allclose(out @ c, f @ c, atol=1e-13)
