"""ctypes binding of the policy in the loop (include/navsim_policy.h).

Argument marshalling only: the actor's forward pass and the steps run in the
library's kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import navsim as _ns

EXPORTS = ("navsim_policy_create", "navsim_policy_layout", "navsim_policy_set_params",
           "navsim_policy_act", "navsim_policy_rollout", "navsim_policy_destroy")
_DONE = False


def _lib():
    global _DONE
    L = _ns.load_library()
    if not _DONE:
        vp, i32, f32 = C.c_void_p, C.c_int32, C.c_float
        L.navsim_policy_create.argtypes = [vp, i32, i32, f32, C.POINTER(vp)]
        L.navsim_policy_layout.argtypes = [vp, vp, vp, vp, vp]
        L.navsim_policy_set_params.argtypes = [vp, vp, C.c_int64]
        L.navsim_policy_act.argtypes = [vp, vp, vp, f32, C.c_uint64, vp]
        L.navsim_policy_rollout.argtypes = [vp, vp, i32, C.c_uint64, vp, f32, vp, vp, vp, vp, vp,
                                            vp, i32, i32, vp]
        L.navsim_policy_destroy.argtypes = [vp]
        for n in EXPORTS:
            getattr(L, n).restype = C.c_int
        _DONE = True
    return L


class Policy:
    """The paper's actor (4 layers, 100 hidden units, leaky ReLU; reciprocal
    range transform with a scalar beta; tanh output) on a NavSim's envs."""

    def __init__(self, sim, hidden: int = 100, hidden_layers: int = 3, leaky_slope: float = 0.01):
        self.sim = sim
        self.device = sim.device
        self.h = None
        h = C.c_void_p()
        _ns._check(_lib().navsim_policy_create(sim.h, int(hidden), int(hidden_layers),
                                               float(leaky_slope), C.byref(h)))
        self.h = h
        self.slope = leaky_slope
        L = C.c_int32()
        cnt = C.c_int64()
        _ns._check(_lib().navsim_policy_layout(self.h, C.byref(L), None, None, C.byref(cnt)))
        dims = (C.c_int32 * (L.value + 1))()
        offs = (C.c_int64 * (2 * L.value + 1))()
        _ns._check(_lib().navsim_policy_layout(self.h, None, dims, offs, None))
        self.dims = list(dims)
        self.offsets = [(offs[2 * l], offs[2 * l + 1]) for l in range(L.value)]
        self.beta_off = offs[2 * L.value]
        self.count = cnt.value

    def close(self):
        h, self.h = getattr(self, "h", None), None
        if h is not None:
            _ns._check(_lib().navsim_policy_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_params(self, seed: int = 0, beta: float = -0.1) -> np.ndarray:
        """Uniform(+-1/sqrt(fan_in)) weights and biases, the given beta."""
        rng = np.random.default_rng(seed)
        p = np.zeros(self.count, np.float32)
        for l, (wo, bo) in enumerate(self.offsets):
            n_in, n_out = self.dims[l], self.dims[l + 1]
            b = 1.0 / np.sqrt(n_in)
            p[wo:wo + n_in * n_out] = rng.uniform(-b, b, n_in * n_out)
            p[bo:bo + n_out] = rng.uniform(-b, b, n_out)
        p[self.beta_off] = beta
        self.set_params(p)
        return p

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _ns._check(_lib().navsim_policy_set_params(self.h, p.ctypes.data, self.count))

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def act(self, obs: torch.Tensor, noise_std: float = 0.0, step: int = 0) -> torch.Tensor:
        _ns._dev_ptr(obs, torch.float32, (self.sim.N, self.sim.m + 4), self.device, "obs")
        a = torch.empty(self.sim.N, 2, dtype=torch.float32, device=self.device)
        _ns._check(_lib().navsim_policy_act(self.h, C.c_void_p(obs.data_ptr()),
                                            C.c_void_p(a.data_ptr()), float(noise_std),
                                            int(step), self._stream()))
        return a

    def rollout(self, steps: int, first_step: int, obs0: torch.Tensor, noise_std: float = 0.0,
                buffers: dict | None = None, kernel: int = _ns.NAVSIM_KERNEL_FUSED,
                graph: bool = True) -> dict:
        b = buffers if buffers is not None else self.sim.rollout_buffers(steps)
        T, N, row = int(steps), self.sim.N, self.sim.m + 4
        dev = self.device
        args = (_ns._dev_ptr(obs0, torch.float32, (N, row), dev, "obs0"),
                _ns._dev_ptr(b["act"], torch.float32, (T, N, 2), dev, "act"),
                _ns._dev_ptr(b["obs"], torch.float32, (T, N, row), dev, "obs"),
                _ns._dev_ptr(b["reward"], torch.float32, (T, N), dev, "reward"),
                _ns._dev_ptr(b["terminated"], torch.uint8, (T, N), dev, "terminated"),
                _ns._dev_ptr(b["truncated"], torch.uint8, (T, N), dev, "truncated"),
                _ns._dev_ptr(b["final_obs"], torch.float32, (T, N, row), dev, "final_obs",
                             optional=True))
        _ns._check(_lib().navsim_policy_rollout(
            self.sim.h, self.h, T, int(first_step), args[0], float(noise_std), *args[1:],
            int(kernel), _ns.NAVSIM_ROLLOUT_GRAPH if graph else 0, self._stream()))
        return b
