"""Pins of the perceptron oracle: bfloat16 rounding against torch's
conversion, backpropagation against central finite differences and against
torch autograd (float64), AdamW against its first-step closed form and
against torch.optim.AdamW."""
import numpy as np
import pytest
import torch

from oracle import mlp as O


def _net(dims, seed=0, slope=0.01):
    rng = np.random.default_rng(seed)
    params = [(rng.normal(0, 1 / np.sqrt(dims[l]), (dims[l + 1], dims[l])),
               rng.normal(0, 0.1, dims[l + 1])) for l in range(len(dims) - 1)]
    return O.MLP(dims, params, slope)


def test_round_bf16_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.uniform(-1e-30, 1e-30, 100),
                        [0.0, -0.0, 1.0, 3e38, -3e38, 1e-45]]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.round_bf16(x), want)
    one = 1.0
    assert O.round_bf16(one + 2.0 ** -8) == 1.0           # tie -> even (1.0)
    assert O.round_bf16(one + 3 * 2.0 ** -8) == one + 2.0 ** -6  # tie -> even (upper)
    assert O.round_bf16(one + 2.0 ** -8 + 2.0 ** -20) == one + 2.0 ** -7
    assert np.isnan(O.round_bf16(np.nan))
    assert O.bf16_bits(1.0) == 0x3F80 and O.from_bf16_bits(0x3F80) == 1.0


def test_backprop_matches_finite_differences():
    dims = [7, 6, 5, 3]
    net = _net(dims, seed=2, slope=0.2)
    rng = np.random.default_rng(3)
    X = rng.normal(size=(9, 7))
    T = rng.normal(size=(9, 3))
    w = np.array([1.0, 0.5, 2.0])
    _, grads = net.loss_grad(X, T, w, emulate=False)
    h = 1e-6
    for l, (W, b) in enumerate(net.params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            for idx in [tuple(np.unravel_index(i, arr.shape)) for i in range(0, arr.size, 3)]:
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = net.loss_grad(X, T, w, emulate=False)
                arr[idx] = old - h
                lm, _ = net.loss_grad(X, T, w, emulate=False)
                arr[idx] = old
                assert abs((lp - lm) / (2 * h) - g[idx]) < 1e-6 * max(1.0, abs(g[idx]))


def test_backprop_matches_torch_autograd():
    dims = [40, 32, 32, 32, 5]
    net = _net(dims, seed=4)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(64, 40))
    T = rng.normal(size=(64, 5))
    w = np.array([1.0, 1.0, 0.0, 1.0, 1.0])
    loss, grads = net.loss_grad(X, T, w, emulate=False)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True))
          for W, b in net.params]
    h = torch.tensor(X)
    for l, (W, b) in enumerate(tp):
        z = h @ W.T + b
        h = torch.nn.functional.leaky_relu(z, net.slope) if l + 1 < len(tp) else z
    tl = ((torch.tensor(w) * (h - torch.tensor(T)) ** 2).sum(1)).mean()
    tl.backward()
    assert abs(tl.item() - loss) < 1e-12
    for (W, b), (gW, gb) in zip(tp, grads):
        assert np.allclose(W.grad.numpy(), gW, rtol=1e-10, atol=1e-13)
        assert np.allclose(b.grad.numpy(), gb, rtol=1e-10, atol=1e-13)


def test_emulated_forward_rounds_only_at_storage_points():
    dims = [16, 8, 4]
    net = _net(dims, seed=6)
    X = np.random.default_rng(7).normal(size=(5, 16))
    Y, hs = net.forward(X, emulate=True)
    assert np.array_equal(hs[0], O.round_bf16(X))
    assert np.array_equal(hs[1], O.round_bf16(hs[1]))
    W2, b2 = net.params[1]
    assert np.allclose(Y, hs[1] @ O.round_bf16(W2).T + b2, rtol=1e-6, atol=1e-6)


def test_adamw_first_step_closed_form_and_torch():
    rng = np.random.default_rng(8)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    decay = np.arange(50) % 3 != 0
    opt = O.AdamW(50, lr=1e-2, wd=0.1, decay=decay)
    p1 = opt.step(p0.copy(), g)
    want = np.where(decay, p0 * (1 - 1e-3), p0) - 1e-2 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p1, want, rtol=1e-12, atol=1e-15)
    # several steps against torch.optim.AdamW (two groups: decayed / not)
    opt = O.AdamW(50, lr=3e-3, wd=0.05, decay=decay)
    p = p0.copy()
    ta = torch.tensor(p0[decay], requires_grad=True)
    tb = torch.tensor(p0[~decay], requires_grad=True)
    topt = torch.optim.AdamW([{"params": [ta], "weight_decay": 0.05},
                              {"params": [tb], "weight_decay": 0.0}], lr=3e-3, eps=1e-8)
    for k in range(6):
        gk = rng.normal(size=50)
        p = opt.step(p, gk)
        ta.grad = torch.tensor(gk[decay])
        tb.grad = torch.tensor(gk[~decay])
        topt.step()
    assert np.allclose(p[decay], ta.detach().numpy(), rtol=1e-12, atol=1e-14)
    assert np.allclose(p[~decay], tb.detach().numpy(), rtol=1e-12, atol=1e-14)
