"""Pins of the actor oracle: the reciprocal input transform and network
against torch (float64), the Box-Muller noise against its closed form on the
KAT-pinned Philox words and against the normal distribution's moments."""
import math

import numpy as np
import torch

import oracle
from oracle import mlp as OM
from oracle import policy as OP


def test_actor_matches_torch():
    rng = np.random.default_rng(0)
    m, H = 30, 100
    dims = [m + 4, H, H, H, 2]
    params = [(rng.normal(0, 1 / math.sqrt(dims[l]), (dims[l + 1], dims[l])),
               rng.normal(0, 0.1, dims[l + 1])) for l in range(4)]
    net = OM.MLP(dims, params, 0.01)
    obs = np.concatenate([rng.uniform(0.0, 6.0, (17, m)), rng.normal(size=(17, 4))], 1)
    beta = -0.25
    x = OP.actor_input(obs, beta, m)
    # the transform: 1 / (l - beta) on the ranges only
    assert np.allclose(x[:, :m], 1.0 / (obs[:, :m] - beta), rtol=1e-6)
    assert np.array_equal(x[:, m:], obs[:, m:].astype(np.float32).astype(np.float64))
    a = OP.actor_forward(net, x, emulate=False)
    h = torch.tensor(x)
    for l, (W, b) in enumerate(params):
        h = h @ torch.tensor(W).T + torch.tensor(b)
        h = torch.nn.functional.leaky_relu(h, net.slope) if l < 3 else torch.tanh(h)
    assert np.allclose(a, h.numpy(), rtol=1e-12, atol=1e-14)
    assert (np.abs(a) < 1).all()


def test_noise_is_box_muller_on_philox_words():
    key = [0x5EED, 0]
    n = OP.noise(6, 12345, key)
    for e in range(6):
        w = oracle.philox4x32_10([e, 12345, 0, 11], key)
        u1, u2 = (w[0] + 0.5) / 2 ** 32, (w[1] + 0.5) / 2 ** 32
        r = math.sqrt(-2 * math.log(u1))
        assert n[e, 0] == r * math.cos(2 * math.pi * u2)
        assert n[e, 1] == r * math.sin(2 * math.pi * u2)
    big = np.concatenate([OP.noise(500, s, key) for s in range(8)]).ravel()
    assert abs(big.mean()) < 0.05 and abs(big.std() - 1.0) < 0.05
    assert abs((np.abs(big) < 1.0).mean() - 0.6827) < 0.03
