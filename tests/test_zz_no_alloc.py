"""The gradient entry point that allocates nothing (lbm_mlp_grad_static, for callers that
cannot call hipMalloc) against lbm_mlp_grad on the same weights and samples, on two calls in a
row, the second with fewer samples: the same kernels in the same order, so the results agree
bit for bit; and its argument checks."""
import numpy as np
import pytest

from gpu_util import announce, require_gpu
from paper_2609_28679_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _samples(n, seed):
    from oracle import mlp
    from oracle.equilibrium import feq
    from oracle.lattice import VARSIGMA2
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.97, 1.03, n)
    u = rng.uniform(-0.06, 0.06, (2, n))
    f = feq(rho, u, VARSIGMA2).T + rng.normal(0.0, 3e-4, (n, 9)) * rho[:, None]
    omega = rng.choice([1 / 0.51, 1 / 0.6, 1.0], n)
    x, _, _ = mlp.features(f, omega)
    return x.astype(np.float32), mlp.targets(f, omega).astype(np.float32)


def test_static_gradient_equals_trainer_gradient_on_two_calls():
    import torch
    from paper_2609_28679_amd import binding as b
    blob = b.pack_mlp(inputs.mlp_init(41))
    w = torch.from_numpy(blob).cuda()
    tr = b.Trainer(blob)
    for n, seed in ((b.MLP_STATIC_MAX_SAMPLES, 42), (3000, 43)):
        announce("lbm_mlp_grad_static n=%d vs lbm_mlp_grad" % n)
        x, t = _samples(n, seed)
        xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
        g_ref = torch.empty(b.MLP_NPARAM, dtype=torch.float32, device="cuda")
        loss_ref = tr.grad(xd, td, g_ref)
        g = torch.full((b.MLP_NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        b.mlp_grad_static(w, xd, td, g, loss)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref), n
        assert float(loss.item()) == loss_ref
        # without the loss output
        g2 = torch.zeros_like(g)
        b.mlp_grad_static(w, xd, td, g2, None)
        torch.cuda.synchronize()
        assert torch.equal(g2, g_ref)
    tr.close()


def test_static_gradient_rejects_sizes_beyond_its_array():
    import torch
    from paper_2609_28679_amd import binding as b
    w = torch.zeros(b.MLP_NPARAM, dtype=torch.float32, device="cuda")
    x = torch.zeros((4, 12), dtype=torch.float32, device="cuda")
    g = torch.zeros(b.MLP_NPARAM, dtype=torch.float32, device="cuda")
    lib = b.load()
    s = b.current_stream_handle()
    too_many = b.MLP_STATIC_MAX_SAMPLES + 1
    assert lib.lbm_mlp_grad_static(w.data_ptr(), x.data_ptr(), x.data_ptr(), too_many,
                                   g.data_ptr(), None, s) == b.LBM_EINVAL
    assert lib.lbm_mlp_grad_static(w.data_ptr(), x.data_ptr(), x.data_ptr(), 0,
                                   g.data_ptr(), None, s) == b.LBM_EINVAL
    assert lib.lbm_mlp_grad_static(None, x.data_ptr(), x.data_ptr(), 4,
                                   g.data_ptr(), None, s) == b.LBM_EINVAL
