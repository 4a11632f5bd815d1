"""Pins of the learned selector's oracle (oracle/mlp_ref.py) against things
other than itself: torch's bf16 conversion, torch's float64 layers, loss and
autograd, central finite differences, torch's Adam, hand-computed features,
and the analytical model of Eq. 1."""
import math
import os

import numpy as np
import pytest
import torch

import graphgen as gg
from oracle import gpop_ref
from oracle import mlp_ref as mr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random_model(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    theta = mr.bf16_round(rng.standard_normal(mr.N_PARAMS).astype(np.float32) * 0.3 * scale)
    mean = rng.standard_normal(12).astype(np.float32)
    inv_std = (0.5 + rng.random(12)).astype(np.float32)
    return theta, mean, inv_std


def _random_batch(seed, n=37):
    rng = np.random.default_rng(seed + 100)
    X = rng.standard_normal((n, 12)).astype(np.float32)
    t_sc = rng.random(n).astype(np.float32) * 10
    t_pc = rng.random(n).astype(np.float32) * 10
    return X, t_sc, t_pc


def _torch_loss(theta, mean, inv_std, X, t_sc, t_pc):
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    P = {
        "W1": th[mr.OFF_W1:mr.OFF_B1].view(64, 12), "b1": th[mr.OFF_B1:mr.OFF_W2],
        "W2": th[mr.OFF_W2:mr.OFF_B2].view(64, 64), "b2": th[mr.OFF_B2:mr.OFF_W3],
        "w3": th[mr.OFF_W3:mr.OFF_B3].view(1, 64), "b3": th[mr.OFF_B3:],
    }
    x = (torch.tensor(X, dtype=torch.float64) - torch.tensor(mean, dtype=torch.float64)) * \
        torch.tensor(inv_std, dtype=torch.float64)
    h = torch.relu(torch.nn.functional.linear(x, P["W1"], P["b1"]))
    h = torch.relu(torch.nn.functional.linear(h, P["W2"], P["b2"]))
    z = torch.nn.functional.linear(h, P["w3"], P["b3"]).view(-1)
    a = torch.tensor(t_sc, dtype=torch.float64)
    b = torch.tensor(t_pc, dtype=torch.float64)
    c = (a - b).abs()
    y = (b < a).to(torch.float64)
    L = torch.nn.functional.binary_cross_entropy_with_logits(z, y, weight=c, reduction="sum") / c.sum()
    L.backward()
    return z.detach().numpy(), L.item(), th.grad.numpy()


def test_param_count_and_layout():
    assert mr.N_PARAMS == 5057
    assert (mr.OFF_B1, mr.OFF_W2, mr.OFF_B2, mr.OFF_W3, mr.OFF_B3) == (768, 832, 4928, 4992, 5056)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.standard_normal(4000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 4000),
        np.array([0.0, -0.0, 1.0, -1.0, 3.4e38, 1e-40, -1e-42, np.inf, -np.inf], np.float32),
    ]).astype(np.float32)
    # exact ties: low half exactly 0x8000 with even and odd upper halves
    u = (rng.integers(0x3F80, 0x4780, 200, dtype=np.uint32) << 16) | 0x8000
    x = np.concatenate([x, u.view(np.float32)])
    ours = mr.bf16_round(x)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_forward_and_loss_match_torch():
    theta, mean, inv_std = _random_model(2)
    X, t_sc, t_pc = _random_batch(2)
    z_ref, L_ref, _ = _torch_loss(theta, mean, inv_std, X, t_sc, t_pc)
    z = mr.forward(theta, mean, inv_std, X)
    L, _ = mr.loss_and_grad(theta, mean, inv_std, X, t_sc, t_pc)
    assert np.allclose(z, z_ref, rtol=1e-12, atol=1e-12)
    assert math.isclose(L, L_ref, rel_tol=1e-12)


def test_inference_forward_matches_torch_bf16_layers():
    """forward_infer against torch: the layer inputs cast to bfloat16 by
    torch (its own round-to-nearest-even conversion), the layers in float64."""
    theta, mean, inv_std = _random_model(6)
    X, _, _ = _random_batch(6, n=211)
    X = X * 3
    W1 = torch.tensor(theta[mr.OFF_W1:mr.OFF_B1], dtype=torch.float64).view(64, 12)
    b1 = torch.tensor(theta[mr.OFF_B1:mr.OFF_W2], dtype=torch.float64)
    W2 = torch.tensor(theta[mr.OFF_W2:mr.OFF_B2], dtype=torch.float64).view(64, 64)
    b2 = torch.tensor(theta[mr.OFF_B2:mr.OFF_W3], dtype=torch.float64)
    w3 = torch.tensor(theta[mr.OFF_W3:mr.OFF_B3], dtype=torch.float64)
    b3 = float(theta[mr.OFF_B3])
    xs = (torch.tensor(X, dtype=torch.float64) - torch.tensor(mean, dtype=torch.float64)) * \
        torch.tensor(inv_std, dtype=torch.float64)
    xb = xs.to(torch.float32).to(torch.bfloat16).to(torch.float64)
    h1 = torch.relu(xb @ W1.T + b1).to(torch.float32).to(torch.bfloat16).to(torch.float64)
    z_ref = (torch.relu(h1 @ W2.T + b2) @ w3 + b3).numpy()
    z = mr.forward_infer(theta, mean, inv_std, X)
    assert np.allclose(z, z_ref, rtol=1e-12, atol=1e-12)
    # and it differs from the exact forward pass by rounding only
    assert 0 < np.max(np.abs(z - mr.forward(theta, mean, inv_std, X))) < 0.05 * np.max(np.abs(z))


def test_inference_forward_is_exact_on_bf16_values():
    """Inputs whose standardised values and first hidden layer are already
    bf16 values (small integers, weights in {-1, 0, 1}): no rounding happens
    and forward_infer equals the exact forward pass."""
    rng = np.random.default_rng(8)
    theta = rng.integers(-1, 2, mr.N_PARAMS).astype(np.float64)
    mean = np.zeros(12, np.float32)
    inv_std = np.ones(12, np.float32)
    X = rng.integers(-3, 4, (50, 12)).astype(np.float32)
    assert np.array_equal(mr.forward_infer(theta, mean, inv_std, X), mr.forward(theta, mean, inv_std, X))


def test_inference_ambiguity_flags_every_rounding_that_moves():
    """Inputs moved by a relative 1e-6 (below the 1e-5 the flag allows for)
    leave forward_infer's roundings, hence its logit, unchanged on every
    sample not flagged ambiguous; the flag marks a minority of samples."""
    theta, mean, inv_std = _random_model(9)
    X, _, _ = _random_batch(9, n=400)
    X = X * 2
    z = mr.forward_infer(theta, mean, inv_std, X)
    amb = mr.infer_ambiguous(theta, mean, inv_std, X)
    assert 0 < np.mean(amb) < 0.5
    rng = np.random.default_rng(10)
    moved = 0
    for _ in range(20):
        Xp = (X * (1 + 1e-6 * rng.standard_normal(X.shape))).astype(np.float64)
        zp = mr.forward_infer(theta, mean, inv_std, Xp)
        d = np.abs(zp - z)
        # unflagged samples: the same bf16 inputs, so the same logit up to the
        # first layer's FP64 sums of slightly different features
        assert np.all(d[~amb] == 0.0)
        moved += int(np.sum(d[amb] > 0))
    assert moved > 0  # some flagged roundings did flip


def test_gradient_matches_torch_autograd():
    theta, mean, inv_std = _random_model(3)
    X, t_sc, t_pc = _random_batch(3, n=53)
    _, _, g_ref = _torch_loss(theta, mean, inv_std, X, t_sc, t_pc)
    _, g = mr.loss_and_grad(theta, mean, inv_std, X, t_sc, t_pc)
    assert np.max(np.abs(g - g_ref)) <= 1e-12 * max(1.0, np.max(np.abs(g_ref)))


def test_gradient_matches_finite_differences():
    theta, mean, inv_std = _random_model(4)
    X, t_sc, t_pc = _random_batch(4, n=29)
    _, g = mr.loss_and_grad(theta, mean, inv_std, X, t_sc, t_pc)
    rng = np.random.default_rng(5)
    idx = list(rng.choice(mr.N_PARAMS, 60, replace=False)) + [mr.OFF_B3, mr.OFF_W3, mr.OFF_B1]
    h = 1e-6
    scale = np.max(np.abs(g))
    for j in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (mr.loss_and_grad(tp, mean, inv_std, X, t_sc, t_pc)[0] -
              mr.loss_and_grad(tm, mean, inv_std, X, t_sc, t_pc)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * scale + 1e-9, j


def test_zero_weight_batch_has_zero_gradient():
    theta, mean, inv_std = _random_model(6)
    X, t_sc, _ = _random_batch(6)
    L, g = mr.loss_and_grad(theta, mean, inv_std, X, t_sc, t_sc)
    assert L == 0.0 and not g.any()


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    theta = rng.standard_normal(50)
    p = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    master, m, v = theta.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        master, m, v = mr.adam_step(master, m, v, g, step, 1e-3)
        assert np.allclose(master, p.detach().numpy(), rtol=0, atol=1e-15)


def test_standardisation_closed_form():
    X = np.array([[1.0, 5.0], [3.0, 5.0]])
    mu, inv = mr.standardisation(X)
    assert np.allclose(mu, [2.0, 5.0])
    assert np.allclose(inv, [1.0, 1e6])


def _golden_graph():
    edges = [(0, 1), (0, 4), (0, 5), (1, 2), (2, 0), (3, 3), (4, 0), (4, 1)]
    n = 6
    off = np.zeros(n + 1, np.uint32)
    for s, _ in edges:
        off[s + 1] += 1
    off = np.cumsum(off).astype(np.uint32)
    cols = np.array([d for _, d in sorted(edges)], np.uint32)
    return off, cols


def test_features_golden():
    off, cols = _golden_graph()
    f = mr.features(off, cols, 4, [0, 4], 3)
    rows = [l.split() for l in open(os.path.join(GOLDEN, "selector_features.txt")) if not l.startswith("#")]
    want = np.array([[float(x) for x in r[1:]] for r in rows])
    assert f.shape == want.shape
    assert np.allclose(f, want, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_last_feature_agrees_with_eq1(seed):
    g = gg.rmat_graph(8, 6, seed=seed)
    q = 32
    rng = np.random.default_rng(seed)
    front = rng.choice(g.n, 70, replace=False)
    f = mr.features(g.offsets, g.cols, q, front, 0)
    png = gpop_ref.build_png(g, q)
    for p in range(png.k):
        va = sum(1 for v in front if v // q == p)
        if va == 0:
            continue
        ea = sum(int(g.offsets[v + 1] - g.offsets[v]) for v in front if v // q == p)
        mode = gpop_ref.choose_mode(png.E[p], png.M[p], va, ea, png.k)
        if abs(f[p, 11] - math.log(2)) > 1e-12:
            assert (f[p, 11] <= math.log(2)) == (mode == gpop_ref.PC)


def test_features_all_active_invariants():
    g = gg.rmat_graph(8, 8, seed=21)
    q = 64
    f = mr.features(g.offsets, g.cols, q, range(g.n), 5)
    assert np.allclose(f[:, 5], 1.0)
    has_edges = f[:, 2] > 0
    assert np.allclose(f[has_edges, 6], 1.0)
    assert np.allclose(f[:, 10], 1.0)
    assert np.allclose(f[:, 9], math.log1p(5))


def test_init_params_shape_and_seed():
    a = gg.mlp_init_params(5)
    b = gg.mlp_init_params(5)
    c = gg.mlp_init_params(6)
    assert a.dtype == np.float32 and a.shape == (5057,)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert not a[mr.OFF_B1:mr.OFF_W2].any() and a[mr.OFF_B3] == 0
