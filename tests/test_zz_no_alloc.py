"""GPU test of the allocation-free gradient entry point (gpop_mlp_grad_noalloc)
through the C-ABI: two calls in a row, the second on a smaller batch, each
against gpop_mlp_grad with a caller workspace on the same inputs (the same
kernels in the same order, so the gradient and loss must agree bit for bit),
and against the FP64 oracle of the gradient; oversized and empty batches are
refused."""
import numpy as np
import pytest

import graphgen as gg
from oracle import mlp_ref as mr
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


def _batch(rng, n):
    X = (rng.standard_normal((n, 12)) * 3).astype(np.float32)
    t_sc = (rng.random(n) * 20).astype(np.float32)
    t_pc = (rng.random(n) * 20).astype(np.float32)
    return X, t_sc, t_pc


def _weights(mlp):
    raw = mlp.model.cpu().numpy().view(np.uint8)
    mean = raw[8:56].view(np.float32).astype(np.float64)
    inv = raw[56:104].view(np.float32).astype(np.float64)
    wbits = raw[104:104 + 2 * 5057].view(np.uint16).astype(np.uint32) << 16
    return mean, inv, wbits.view(np.float32).astype(np.float64)


def test_noalloc_gradient_equals_workspace_gradient_twice():
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    rng = np.random.default_rng(2024)
    mlp = gp.Mlp()
    X0, _, _ = _batch(rng, 4096)
    mlp.init(torch.from_numpy(gg.mlp_init_params(5)).cuda(), torch.from_numpy(X0).cuda())
    mean, inv, w = _weights(mlp)
    # the largest batch the fixed array takes, then a smaller ragged one
    for n in (gp.MLP_NOALLOC_MAX_SAMPLES, 1000):
        print("noalloc gradient n =", n, flush=True)
        X, t_sc, t_pc = _batch(rng, n)
        xt, at, bt = (torch.from_numpy(a).cuda() for a in (X, t_sc, t_pc))
        g_ws = mlp.compute_grad(xt, at, bt).clone()
        l_ws = mlp.loss.clone()
        g_na = torch.full_like(g_ws, float("nan"))
        l_na = torch.full_like(l_ws, float("nan"))
        mlp.compute_grad_noalloc(xt, at, bt, grad=g_na, loss=l_na)
        torch.cuda.synchronize()
        assert torch.equal(g_na, g_ws), n
        assert torch.equal(l_na, l_ws), n
        L, gr = mr.loss_and_grad(w, mean, inv, X, t_sc, t_pc)
        g = g_na.cpu().numpy()
        assert abs(float(l_na[0]) - L) <= 1e-4 * max(1.0, abs(L))
        assert np.max(np.abs(g - gr)) / max(np.max(np.abs(gr)), 1e-30) <= 1e-3


def test_noalloc_gradient_rejects_sizes():
    torch = torch_cuda()
    import paper_1806_08092_amd as gp
    mlp = gp.Mlp()
    rng = np.random.default_rng(7)
    X, t_sc, t_pc = _batch(rng, gp.MLP_NOALLOC_MAX_SAMPLES + 1)
    mlp.init(torch.from_numpy(gg.mlp_init_params(6)).cuda(), torch.from_numpy(X).cuda())
    xt, at, bt = (torch.from_numpy(a).cuda() for a in (X, t_sc, t_pc))
    with pytest.raises(gp.GpopError) as e:
        mlp.compute_grad_noalloc(xt, at, bt)
    assert e.value.code == gp.EINVAL and "GPOP_MLP_NOALLOC_MAX_SAMPLES" in str(e.value)
    with pytest.raises(gp.GpopError) as e:
        mlp.compute_grad_noalloc(xt[:0], at[:0], bt[:0])
    assert e.value.code == gp.EINVAL
