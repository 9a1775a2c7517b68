"""Oracle of the actor in the loop (TEST INFRASTRUCTURE ONLY): the state of
eq. 1 with the reciprocal range transform of eq. 2, a perceptron with leaky
ReLU hidden layers (section 2.1) and a tanh output, in float64, optionally
rounding to bfloat16 where the GPU stores bfloat16; and the exploration noise
(Box-Muller on Philox words)."""
from __future__ import annotations

import math

import numpy as np

from . import philox4x32_10
from .mlp import MLP, round_bf16


def actor_input(obs, beta: float, m: int) -> np.ndarray:
    """[l_1..l_m, d, phi, v, w] -> [1 / (l_j - beta), d, phi, v, w], float32 as
    the GPU computes it (one float32 division)."""
    o = np.asarray(obs, np.float32)
    x = o.copy()
    x[:, :m] = (np.float32(1.0) / (o[:, :m] - np.float32(beta))).astype(np.float32)
    return x.astype(np.float64)


def actor_forward(net: MLP, x, emulate: bool = True) -> np.ndarray:
    """Hidden layers leaky ReLU, output tanh."""
    y, _ = net.forward(x, emulate=emulate)
    return np.tanh(y)


def noise(N: int, step: int, key) -> np.ndarray:
    """Standard normal pairs per env: Box-Muller on Philox(e, step lo, step hi,
    11) words 0 and 1, u = (w + 1/2) 2^-32."""
    out = np.zeros((N, 2))
    for e in range(N):
        w = philox4x32_10([e, step & 0xFFFFFFFF, (step >> 32) & 0xFFFFFFFF, 11], key)
        u1, u2 = (w[0] + 0.5) / 2 ** 32, (w[1] + 0.5) / 2 ** 32
        r, t = math.sqrt(-2.0 * math.log(u1)), 2.0 * math.pi * u2
        out[e] = (r * math.cos(t), r * math.sin(t))
    return out


def policy_params(flat, dims, offsets):
    return MLP.unflatten(dims, np.asarray(flat, np.float64), offsets)
