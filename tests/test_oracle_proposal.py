"""Pins of the proposal-network oracle: convolutions against torch's FP64 conv2d (a library
routine for the same definition), gradients by finite differences and against torch
autograd, BF16 rounding against known values and torch's conversion, Adam against torch."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import proposal as P


def torch_conv(x, w, b, stride, up):
    xt = torch.tensor(x).permute(2, 0, 1)[None]
    if up:
        xt = F.interpolate(xt, scale_factor=2, mode="nearest")
    y = F.conv2d(xt, torch.tensor(w).permute(0, 3, 1, 2), torch.tensor(b), stride=stride, padding=1)
    return y[0].permute(1, 2, 0).numpy()


@pytest.mark.parametrize("H,W,stride,up", [(7, 9, 1, False), (7, 9, 2, False), (8, 6, 2, False), (5, 6, 1, True)])
def test_conv_matches_torch(H, W, stride, up):
    rng = np.random.default_rng(1)
    x = rng.normal(size=(H, W, 5))
    w = rng.normal(size=(4, 3, 3, 5))
    b = rng.normal(size=4)
    np.testing.assert_allclose(P.conv3x3(x, w, b, stride, up), torch_conv(x, w, b, stride, up), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("stride,up", [(1, False), (2, False), (1, True)])
def test_conv_backward_matches_autograd(stride, up):
    rng = np.random.default_rng(2)
    x = rng.normal(size=(6, 7, 3))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = P.conv3x3(x, w, b, stride, up)
    dy = rng.normal(size=y.shape)
    dx, dw, db = P.conv3x3_backward(x, w, dy, stride, up)
    xt, wt, bt = (torch.tensor(a, requires_grad=True) for a in (x, w, b))
    xi = xt.permute(2, 0, 1)[None]
    if up:
        xi = F.interpolate(xi, scale_factor=2, mode="nearest")
    yt = F.conv2d(xi, wt.permute(0, 3, 1, 2), bt, stride=stride, padding=1)[0].permute(1, 2, 0)
    (yt * torch.tensor(dy)).sum().backward()
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dw, wt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


def tiny_problem(seed=3, H=6, W=8, N=2):
    rng = np.random.default_rng(seed)
    params = P.init_params(seed, N)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng.normal(scale=0.1, size=params[k].shape)
    flow = rng.normal(scale=8.0, size=(N, H, W, 2))
    rho_t = rng.uniform(0.05, 0.5, size=(H, W))
    q_t = rng.uniform(0, 1, size=(N, H, W))
    mask = rng.uniform(size=(H, W)) < 0.8
    return params, P.features(flow), rho_t, q_t, mask


def total_loss(params, x, rho_t, q_t, mask):
    return P.loss(P.forward(params, x)["o"], rho_t, q_t, 1.3, mask, 0.5)[0]


def test_network_gradient_by_finite_differences():
    params, x, rho_t, q_t, mask = tiny_problem()
    acts = P.forward(params, x)
    L, do = P.loss(acts["o"], rho_t, q_t, 1.3, mask, 0.5)
    grads = P.backward(params, acts, do)
    rng = np.random.default_rng(4)
    for name in ("c1.w", "c2.w", "c3.b", "c4.w", "c5.w", "c5.b", "c6.w", "c6.b"):
        flat = np.flatnonzero(np.abs(params[name]).ravel() > 0) if name.endswith(".w") else np.arange(params[name].size)
        for idx in rng.choice(flat, size=3, replace=False):
            p2 = {k: v.copy() for k, v in params.items()}
            h = 1e-6
            p2[name].ravel()[idx] += h
            Lp = total_loss(p2, x, rho_t, q_t, mask)
            p2[name].ravel()[idx] -= 2 * h
            Lm = total_loss(p2, x, rho_t, q_t, mask)
            fd = (Lp - Lm) / (2 * h)
            assert grads[name].ravel()[idx] == pytest.approx(fd, rel=1e-4, abs=1e-9), (name, idx)


def test_heads_and_loss_limits():
    o = np.zeros((2, 3, P.C_HEAD))
    rho, q = P.heads(o, 2, 2.0, 0.01, 1.0)
    np.testing.assert_allclose(rho, np.log(2) / 2)
    np.testing.assert_allclose(q, 0.5)
    # perfect depth and q = 0.5 targets: L1 part 0, BCE part log 2
    L, do = P.loss(o, np.full((2, 3), np.log(2) / 2), np.full((2, 2, 3), 0.5), 2.0, np.ones((2, 3), bool), 1.0)
    assert L == pytest.approx(np.log(2))
    assert np.all(do[..., 1:3] == 0)


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8 - 2 ** -20, 3.14159, 1e-40, 65504.0, np.inf])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, -1 - 2 ** -7, 3.140625, None, 65536.0, np.inf], dtype=object)
    got = P.bf16(vals)
    for g, wv in zip(got, want):
        if wv is not None:
            assert g == wv
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(got, ref)
    rng = np.random.default_rng(5)
    r = rng.normal(scale=10.0, size=10000)
    np.testing.assert_array_equal(P.bf16(r), torch.tensor(r, dtype=torch.float32).to(torch.bfloat16).double().numpy())


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    params = {"a": rng.normal(size=(3, 4)), "b": rng.normal(size=5)}
    tp = {k: torch.tensor(v.copy(), requires_grad=True) for k, v in params.items()}
    opt = torch.optim.Adam(tp.values(), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = {k: np.zeros_like(v) for k, v in params.items()}
    v = {k: np.zeros_like(x) for k, x in params.items()}
    for step in range(1, 4):
        grads = {k: rng.normal(size=x.shape) for k, x in params.items()}
        P.adam_step(params, grads, m, v, step, 1e-3)
        for k in tp:
            tp[k].grad = torch.tensor(grads[k])
        opt.step()
    for k in params:
        np.testing.assert_allclose(params[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-14)


def test_param_count():
    params = P.init_params(0, 6)
    real = sum(int(np.count_nonzero(v)) for k, v in params.items() if k.endswith(".w"))
    real += sum(co for _, _, co, _, _, _, _ in P.LAYERS[:-1]) + 7
    assert 440_000 < real < 470_000
