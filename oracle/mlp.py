"""Oracle of the reset proposal's perceptron (TEST INFRASTRUCTURE ONLY).

Plain numpy in float64: dense layers y = x W^T + b, leaky ReLU between them,
a weighted squared-error loss, backpropagation written out layer by layer,
and AdamW with decoupled weight decay (Loshchilov & Hutter, ICLR'19).

``emulate=True`` rounds to bfloat16 at the points where the GPU kernels store
bfloat16 (weights, inputs, hidden activations, the backward pass's layer
gradients before they enter a product), so that what remains between the two
sides is float32 versus float64 accumulation.  ``emulate=False`` is the exact
real-number network, which the finite-difference and autograd pins check.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x) -> np.ndarray:
    """Nearest bfloat16 value (ties to even) of float32(x), as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def bf16_bits(x) -> np.ndarray:
    """uint16 bit patterns of round_bf16(x)."""
    v = round_bf16(x).astype(np.float32).view(np.uint32) >> 16
    return v.astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, np.uint32) << 16).view(np.float32).astype(np.float64)


def leaky(z, slope):
    return np.where(z > 0, z, slope * z)


class MLP:
    """dims = [d0, d1, ..., dL]; leaky ReLU after every layer but the last.
    params: list of (W [d_{l+1}, d_l], b [d_{l+1}]) in float64."""

    def __init__(self, dims, params, slope: float = 0.01):
        self.dims = list(dims)
        self.params = [(np.array(W, np.float64), np.array(b, np.float64)) for W, b in params]
        self.slope = float(np.float32(slope))

    @staticmethod
    def unflatten(dims, flat, offsets):
        """offsets: [(w_off, b_off)] per layer into the flat float vector."""
        out = []
        for l in range(len(dims) - 1):
            wo, bo = offsets[l]
            n_out, n_in = dims[l + 1], dims[l]
            out.append((np.array(flat[wo:wo + n_out * n_in], np.float64).reshape(n_out, n_in),
                        np.array(flat[bo:bo + n_out], np.float64)))
        return out

    def forward(self, X, emulate: bool = True):
        """Returns (Y, hs): outputs and the inputs of each layer."""
        r = round_bf16 if emulate else (lambda a: np.asarray(a, np.float64))
        h = r(X)
        hs = [h]
        L = len(self.params)
        for l, (W, b) in enumerate(self.params):
            z = h @ r(W).T + b
            if l + 1 < L:
                h = r(leaky(z, self.slope))
                hs.append(h)
            else:
                y = z.astype(np.float32).astype(np.float64) if emulate else z
        return y, hs

    def loss_grad(self, X, T, w, emulate: bool = True):
        """Mean over rows of sum_d w_d (y - t)^2, and its gradient with respect
        to every (W, b)."""
        r = round_bf16 if emulate else (lambda a: np.asarray(a, np.float64))
        Y, hs = self.forward(X, emulate)
        M = Y.shape[0]
        E = Y - np.asarray(T, np.float64)
        w = np.asarray(w, np.float64)
        loss = (w * E * E).sum(axis=1).mean()
        dz = 2.0 * w * E / M
        if emulate:
            dz = dz.astype(np.float32).astype(np.float64)
        grads = [None] * len(self.params)
        for l in range(len(self.params) - 1, -1, -1):
            W, _ = self.params[l]
            dzr = r(dz)
            grads[l] = (dzr.T @ hs[l], dz.sum(axis=0))
            if l == 0:
                break
            dh = dzr @ r(W)
            deriv = np.where(hs[l] > 0, 1.0, self.slope)
            dz = dh * deriv
            if emulate:
                dz = dz.astype(np.float32).astype(np.float64)
        return loss, grads


class AdamW:
    """p <- p (1 - lr wd) - lr m_hat / (sqrt(v_hat) + eps), moments as in
    Adam; weight decay only where decay[i] is true."""

    def __init__(self, n, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0, decay=None):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps, self.wd = lr, b1, b2, eps, wd
        self.decay = np.ones(n, bool) if decay is None else np.asarray(decay, bool)

    def step(self, p, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        p = np.where(self.decay, p * (1 - self.lr * self.wd), p)
        return p - self.lr * mh / (np.sqrt(vh) + self.eps)
