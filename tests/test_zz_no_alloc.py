"""The allocation-free gradient entry point (ovl_mlp_gradient_static) against
the trainer's gradient (ovl_mlp_gradient), through the C ABI.

Both run the same kernels on the same rows, so the gradient and the loss must
agree bit for bit.  Two calls in a row, the second on fewer rows than the
first: the fixed partial-result array then still holds the first call's extra
blocks, which the second call must not read.  Sizes above the fixed array's
room are rejected before anything is queued.
"""
import numpy as np
import pytest

import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes

pytestmark = pytest.mark.gpu


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 12)).astype(np.float32)
    t = rng.standard_normal((n, 3)).astype(np.float32)
    return x, t


def test_static_gradient_matches_trainer_gradient():
    import torch

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    params = scenes.mlp_initial_weights(3)
    tr = ovl.Trainer(params)
    p_d = torch.from_numpy(params).to(dev)
    grad_d = torch.full((ovl.MLP_PARAMS,), float("nan"), device=dev)
    loss_d = torch.full((1,), float("nan"), device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    for n, seed in ((5000, 11), (700, 12), (ovl.MLP_STATIC_ROWS, 13)):
        x, t = _rows(n, seed)
        ref_loss, ref_grad = tr.gradient(x, t)
        x_d = torch.from_numpy(x).to(dev)
        t_d = torch.from_numpy(t).to(dev)
        ovl.ovl_mlp_gradient_static(p_d, x_d, t_d, grad_d, loss_d, stream)
        torch.cuda.synchronize()
        g = grad_d.cpu().numpy()
        loss = float(loss_d.cpu().numpy()[0])
        assert np.array_equal(g, ref_grad), (n, float(np.abs(g - ref_grad).max()))
        assert np.float32(loss) == np.float32(ref_loss), (n, loss, ref_loss)
        assert np.isfinite(g).all() and loss > 0.0
    tr.close()


def test_static_gradient_rejects_sizes_beyond_its_array():
    import torch

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    n = ovl.MLP_STATIC_ROWS + 1
    p_d = torch.zeros(ovl.MLP_PARAMS, device=dev)
    x_d = torch.zeros((n, 12), device=dev)
    t_d = torch.zeros((n, 3), device=dev)
    grad_d = torch.zeros(ovl.MLP_PARAMS, device=dev)
    loss_d = torch.zeros(1, device=dev)
    with pytest.raises(ovl.OvlError, match="OVL_MLP_STATIC_ROWS"):
        ovl.ovl_mlp_gradient_static(p_d, x_d, t_d, grad_d, loss_d)
    torch.cuda.synchronize()
    assert float(grad_d.abs().sum()) == 0.0          # nothing was queued
