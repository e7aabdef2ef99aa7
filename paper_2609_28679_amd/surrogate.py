"""Training-data harvest and training of the learned collision surrogate (host orchestration).

Every numerical step runs in the library: lbm_step advances the paper's scheme, lbm_harvest
writes network inputs and plain-collision targets for chosen nodes, lbm_mlp_train runs the
bfloat16 forward/backward/Adam kernels. This module only sequences those calls and moves
seeded node lists to the device.
"""
import numpy as np

from . import binding, inputs


def harvest(fields, taus, n_samples, step_range, n_harvests, seed, **lattice_kw):
    """Run one D2Q9 isothermal lattice per tau from `fields` = (rho, u) and harvest
    n_samples // (len(taus) * n_harvests) random nodes at n_harvests steps spread evenly over
    step_range = (first, last). Returns device tensors X (N, 12) and Y (N, 9)."""
    import torch
    rho, u = fields
    nodes = rho.size
    steps = np.linspace(step_range[0], step_range[1], n_harvests).round().astype(np.int64)
    per_tau = n_samples // len(taus)
    xs, ys = [], []
    for k, tau in enumerate(taus):
        plan = inputs.harvest_plan(nodes, per_tau, list(steps), seed + 1000 * k)
        lat = binding.Lattice(rho, u, tau=tau, **lattice_kw)
        for s, idx in plan:
            lat.step(s - lat.t)
            n = len(idx)
            d_idx = torch.from_numpy(idx).cuda()
            X = torch.empty((n, 12), dtype=torch.float32, device="cuda")
            Y = torch.empty((n, 9), dtype=torch.float32, device="cuda")
            lat.harvest(d_idx, X, Y)
            xs.append(X)
            ys.append(Y)
        lat.close()
    return torch.cat(xs), torch.cat(ys)


def shuffle(X, Y, seed):
    """Seeded permutation of the samples (applied on the device)."""
    import torch
    perm = np.random.default_rng(seed).permutation(X.shape[0])
    p = torch.from_numpy(perm).cuda()
    return X[p].contiguous(), Y[p].contiguous()


def train(X, Y, init_params, batch=4096, steps=4000, lr=1e-3, schedule=None):
    """Adam on the MSE loss; returns (trainer, float32 weight blob). `schedule`, a list of
    (steps, lr) stages run in order with the Adam state carried over, replaces steps and lr."""
    tr = binding.Trainer(binding.pack_mlp(init_params))
    for n, rate in (schedule or [(steps, lr)]):
        tr.train(X, Y, batch, n, rate)
    return tr, tr.weights()


def loss(trainer, X, Y):
    import torch
    g = torch.empty(binding.MLP_NPARAM, dtype=torch.float32, device="cuda")
    return trainer.grad(X, Y, g)
