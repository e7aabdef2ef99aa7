"""Reference for the learned collision surrogate (not part of the paper's method: the paper's
collision of Eq. (LBM_f) is the judge of its error and its fallback).

Network (D2Q9): 12 inputs -> 64 (GELU) -> 64 (GELU) -> 9 outputs, followed by an exact
projection of the 9 outputs onto the subspace with zero mass and zero momentum, so that the
predicted post-collision populations keep the node's rho and rho u (the invariants of the
paper's collision, Sec. II C).

Encoding per node, with f^eq the paper's product-form equilibrium at theta = 1/3:
  inputs   x = [S (f_i - f_i^eq)/rho  (i = 0..8),  U u_x,  U u_y,  omega]
  target   t = S (f~_i - f_i^eq)/rho   (f~ the plain collision of Eq. (LBM_f))
  decode   f~_i = f_i^eq + rho * y_i / S
with S = 1024 and U = 16 (powers of two, so scaling is exact in any binary format).

GELU is the tanh form of Hendrycks and Gimpel (2016):
  gelu(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).
Loss: mean squared error over batch and outputs. Optimiser: Adam (Kingma and Ba, 2015) with
bias correction.

All arithmetic is float64. `bf16=True` rounds the operands of every matrix product to
bfloat16 (round to nearest even), to mirror a BF16 matrix-core implementation that
accumulates in higher precision.
"""
import numpy as np

from .equilibrium import feq
from .lattice import VARSIGMA2, velocities

S_NEQ = 1024.0
S_U = 16.0
N_IN, N_HID, N_OUT = 12, 64, 9
GELU_K = np.sqrt(2.0 / np.pi)
GELU_A = 0.044715


def round_bf16(x):
    """Round to the nearest bfloat16 (ties to even); returns float64 holding the value."""
    x32 = np.asarray(x, dtype=np.float32)
    bits = x32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = rounded.view(np.float32).astype(np.float64)
    # NaN/inf pass through unchanged
    nonfinite = ~np.isfinite(x32)
    out[nonfinite] = x32[nonfinite]
    return out


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_K * (z + GELU_A * z ** 3)))


def gelu_grad(z):
    t = np.tanh(GELU_K * (z + GELU_A * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_K * (1.0 + 3.0 * GELU_A * z * z)


def constraint_matrix():
    """Rows: 1, c_x, c_y over the 9 directions."""
    c = velocities(2).astype(np.float64)
    return np.stack([np.ones(9), c[:, 0], c[:, 1]])


def project(y):
    """Orthogonal projection of y (batch, 9) onto {y : C y = 0}."""
    C = constraint_matrix()
    return y - (y @ C.T) @ np.linalg.solve(C @ C.T, C)


def features(f, omega):
    """Inputs x (N, 12) and f^eq (N, 9), rho (N,) from pre-collision f (N, 9)."""
    c = velocities(2).astype(np.float64)
    rho = f.sum(axis=1)
    u = (f @ c) / rho[:, None]
    fe = feq(rho, u.T, VARSIGMA2).T
    x = np.empty((f.shape[0], N_IN))
    x[:, :9] = S_NEQ * (f - fe) / rho[:, None]
    x[:, 9] = S_U * u[:, 0]
    x[:, 10] = S_U * u[:, 1]
    x[:, 11] = omega
    return x, fe, rho


def targets(f, omega):
    """S (f~ - f^eq)/rho for the plain collision f~ = f + omega (f^eq - f)."""
    _, fe, rho = features(f, omega)
    ft = f + np.asarray(omega).reshape(-1, 1) * (fe - f)
    return S_NEQ * (ft - fe) / rho[:, None]


def forward(params, x, bf16=False):
    """Returns output y (projected) and the cache needed by backward."""
    W1, b1, W2, b2, W3, b3 = params
    r = round_bf16 if bf16 else (lambda a: a)
    x0 = r(x)
    z1 = x0 @ r(W1).T + b1
    h1 = r(gelu(z1))
    z2 = h1 @ r(W2).T + b2
    h2 = r(gelu(z2))
    y = h2 @ r(W3).T + b3
    return project(y), (x0, z1, h1, z2, h2)


def loss(yhat, t):
    return np.mean((yhat - t) ** 2)


def backward(params, cache, yhat, t, bf16=False):
    """Gradients of the MSE loss with respect to W1, b1, W2, b2, W3, b3."""
    W1, b1, W2, b2, W3, b3 = params
    r = round_bf16 if bf16 else (lambda a: a)
    x0, z1, h1, z2, h2 = cache
    B = t.shape[0]
    dyhat = 2.0 * (yhat - t) / (B * N_OUT)
    dy = project(dyhat)              # the projection is symmetric
    dy_r = r(dy)
    dW3 = dy_r.T @ h2
    db3 = dy.sum(axis=0)
    dh2 = dy_r @ r(W3)
    dz2 = dh2 * gelu_grad(z2)
    dz2_r = r(dz2)
    dW2 = dz2_r.T @ h1
    db2 = dz2.sum(axis=0)
    dh1 = dz2_r @ r(W2)
    dz1 = dh1 * gelu_grad(z1)
    dz1_r = r(dz1)
    dW1 = dz1_r.T @ x0
    db1 = dz1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]


class Adam:
    def __init__(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m = None
        self.v = None

    def step(self, params, grads):
        if self.m is None:
            self.m = [np.zeros_like(p) for p in params]
            self.v = [np.zeros_like(p) for p in params]
        self.t += 1
        out = []
        for k, (p, g) in enumerate(zip(params, grads)):
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * g * g
            mhat = self.m[k] / (1.0 - self.b1 ** self.t)
            vhat = self.v[k] / (1.0 - self.b2 ** self.t)
            out.append(p - self.lr * mhat / (np.sqrt(vhat) + self.eps))
        return out


def surrogate_collide(params, f, omega, tol, bf16=False):
    """Post-collision populations of the surrogate with per-node fallback to the plain
    collision when |f~_mlp - f~_plain| > tol |f~_plain - f^eq| (Euclidean norms over i).

    f: (N, 9) pre-collision populations. Returns (f~, fallback mask).
    """
    x, fe, rho = features(f, omega)
    y, _ = forward(params, x, bf16)
    f_mlp = fe + rho[:, None] * y / S_NEQ
    f_plain = f + np.asarray(omega).reshape(-1, 1) * (fe - f)
    err = np.sqrt(((f_mlp - f_plain) ** 2).sum(axis=1))
    ref = np.sqrt(((f_plain - fe) ** 2).sum(axis=1))
    fallback = err > tol * ref
    out = np.where(fallback[:, None], f_plain, f_mlp)
    return out, fallback
