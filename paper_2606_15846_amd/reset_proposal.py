"""ctypes binding of the learned reset proposal (include/navsim_reset_proposal.h).

Argument marshalling only: labelling, training, proposing and the network run
in the library's kernels.  Device arrays are torch tensors on the simulator's
device.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import navsim as _ns

EXPORTS = ("navsim_rp_create", "navsim_rp_label", "navsim_rp_train", "navsim_rp_propose",
           "navsim_rp_propose_noalloc", "navsim_rp_forward", "navsim_rp_loss_grad",
           "navsim_rp_adamw", "navsim_rp_layout",
           "navsim_rp_get_params", "navsim_rp_set_params", "navsim_rp_destroy",
           "navsim_rp_attach", "navsim_rp_detach", "navsim_rp_attach_stats",
           "navsim_rp_attach_outputs")
STAT_NAMES = ("deferred", "over_cap", "requests", "from_network", "from_rejection", "no_pair",
              "checks")


class RPConfig(C.Structure):
    _fields_ = [("num_bins", C.c_int32), ("d_lo_m", C.c_float), ("d_hi_m", C.c_float),
                ("noise_dim", C.c_int32), ("hidden", C.c_int32), ("hidden_layers", C.c_int32),
                ("leaky_slope", C.c_float), ("seed", C.c_uint64)]


DEFAULT = dict(num_bins=8, d_lo_m=1.0, d_hi_m=12.0, noise_dim=16, hidden=256, hidden_layers=3,
               leaky_slope=0.01, seed=0xC0FFEE)

_DONE = False


def _lib():
    global _DONE
    L = _ns.load_library()
    if not _DONE:
        vp, i32, i64, f32, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_uint32
        L.navsim_rp_create.argtypes = [vp, C.POINTER(RPConfig), C.POINTER(vp)]
        L.navsim_rp_label.argtypes = [vp, i32, vp, u32, vp, vp, vp, vp]
        L.navsim_rp_train.argtypes = [vp, i32, vp, vp, vp, vp, i32, i32, i32, f32, f32, vp, vp]
        L.navsim_rp_propose.argtypes = [vp, i32, vp, vp, vp, vp, i32, i32, vp, vp, vp, vp, vp, vp]
        L.navsim_rp_propose_noalloc.argtypes = L.navsim_rp_propose.argtypes
        L.navsim_rp_forward.argtypes = [vp, i32, vp, vp, vp]
        L.navsim_rp_loss_grad.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.navsim_rp_adamw.argtypes = [vp, vp, f32, f32, vp]
        L.navsim_rp_layout.argtypes = [vp, vp, vp, vp, vp]
        L.navsim_rp_get_params.argtypes = [vp, vp, i64]
        L.navsim_rp_set_params.argtypes = [vp, vp, i64]
        L.navsim_rp_destroy.argtypes = [vp]
        L.navsim_rp_attach.argtypes = [vp, vp, i32, i32, i32]
        L.navsim_rp_detach.argtypes = [vp]
        L.navsim_rp_attach_stats.argtypes = [vp, vp, i32]
        L.navsim_rp_attach_outputs.argtypes = [vp, vp, vp, vp]
        for n in EXPORTS:
            getattr(L, n).restype = C.c_int
        _DONE = True
    return L


def _ptr(t, dtype=None, optional=False, name="array"):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


class ResetProposer:
    """Learned reset proposal over the maps loaded in a NavSim."""

    def __init__(self, sim, **cfg):
        c = dict(DEFAULT)
        c.update(cfg)
        self.cfg = c
        self.sim = sim
        self.device = sim.device
        self.h = None
        rc = RPConfig(**{k: c[k] for k, _ in RPConfig._fields_})
        h = C.c_void_p()
        _ns._check(_lib().navsim_rp_create(sim.h, C.byref(rc), C.byref(h)))
        self.h = h
        sim._proposers.add(self)
        self.nb = int(c["num_bins"])
        L = C.c_int32()
        cnt = C.c_int64()
        _ns._check(_lib().navsim_rp_layout(self.h, C.byref(L), None, None, C.byref(cnt)))
        dims = (C.c_int32 * (L.value + 1))()
        offs = (C.c_int64 * (2 * L.value))()
        _ns._check(_lib().navsim_rp_layout(self.h, None, dims, offs, None))
        self.dims = list(dims)
        self.offsets = [(offs[2 * l], offs[2 * l + 1]) for l in range(L.value)]
        self.count = cnt.value
        self.d0 = self.dims[0]

    def close(self):
        h, self.h = getattr(self, "h", None), None
        if h is not None:
            _ns._check(_lib().navsim_rp_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def label(self, map_ids, first_sid: int) -> dict:
        m = torch.as_tensor(np.asarray(map_ids, np.int32), device=self.device)
        n = m.numel()
        z = dict(dtype=torch.int32, device=self.device)
        out = dict(start=torch.empty(n, **z), goal=torch.empty(n, self.nb, **z),
                   hops=torch.empty(n, self.nb, **z))
        _ns._check(_lib().navsim_rp_label(self.h, n, _ptr(m), int(first_sid) & 0xFFFFFFFF,
                                          _ptr(out["start"]), _ptr(out["goal"]),
                                          _ptr(out["hops"]), self._stream()))
        return out

    def train(self, pairs: dict, steps: int, batch: int = 1024, samples: int = 16,
              lr: float = 1e-3, weight_decay: float = 1e-4, loss=None):
        """pairs: device int32 tensors map, bin, start, goal of equal length."""
        n = pairs["map"].numel()
        _ns._check(_lib().navsim_rp_train(
            self.h, n, _ptr(pairs["map"], torch.int32), _ptr(pairs["bin"], torch.int32),
            _ptr(pairs["start"], torch.int32), _ptr(pairs["goal"], torch.int32), int(steps),
            int(batch), int(samples), float(lr), float(weight_decay),
            _ptr(loss, torch.float32, optional=True), self._stream()))

    def propose(self, map_ids, bins, env, episode, proposals: int, max_tries: int,
                want_y: bool = False, noalloc: bool = False) -> dict:
        """noalloc: the entry point that takes its workspace from the fixed
        per-device array (navsim_rp_propose_noalloc) instead of allocating."""
        dev = self.device
        m = torch.as_tensor(map_ids, dtype=torch.int32, device=dev).contiguous()
        b = torch.as_tensor(bins, dtype=torch.int32, device=dev).contiguous()
        e = torch.as_tensor(np.asarray(env, np.uint32).view(np.int32), device=dev).contiguous()
        ep = torch.as_tensor(np.asarray(episode, np.uint32).view(np.int32), device=dev).contiguous()
        n = m.numel()
        z = dict(device=dev)
        out = dict(pose=torch.empty(n, 5, dtype=torch.float32, **z),
                   hops=torch.empty(n, dtype=torch.int32, **z),
                   source=torch.empty(n, dtype=torch.int32, **z),
                   checks=torch.empty(n, dtype=torch.int32, **z))
        if want_y and proposals > 0:
            out["y"] = torch.empty(n, proposals, 5, dtype=torch.float32, **z)
        return self.propose_into(m, b, e, ep, proposals, max_tries, out, noalloc=noalloc)

    def propose_into(self, m, b, e, ep, proposals, max_tries, out, noalloc: bool = False):
        n = m.numel()
        fn = _lib().navsim_rp_propose_noalloc if noalloc else _lib().navsim_rp_propose
        _ns._check(fn(
            self.h, n, _ptr(m), _ptr(b), _ptr(e), _ptr(ep), int(proposals), int(max_tries),
            _ptr(out["pose"]), _ptr(out["hops"]), _ptr(out["source"]), _ptr(out["checks"]),
            _ptr(out.get("y"), optional=True), self._stream()))
        return out

    def attach(self, bins, proposals: int, max_tries: int, max_per_step: int):
        """Learned resets inside NavSim.step / reset for envs with bins[e] >= 0
        (navsim_rp_attach); bins: int [num_envs], -1 = free-space sampler."""
        b = np.ascontiguousarray(np.asarray(bins, np.int32))
        if b.shape != (self.sim.N,):
            raise ValueError(f"bins must have shape ({self.sim.N},)")
        _ns._check(_lib().navsim_rp_attach(self.h, b.ctypes.data, int(proposals),
                                           int(max_tries), int(max_per_step)))

    def detach(self):
        _ns._check(_lib().navsim_rp_detach(self.h))

    def attach_stats(self, clear: bool = False) -> dict:
        out = np.zeros(8, np.int64)
        _ns._check(_lib().navsim_rp_attach_stats(self.h, out.ctypes.data, int(bool(clear))))
        return {k: int(v) for k, v in zip(STAT_NAMES, out)}

    def attach_outputs(self) -> tuple[torch.Tensor, torch.Tensor]:
        """(source, hops) per env of the last step or reset (device int32 [N])."""
        z = dict(dtype=torch.int32, device=self.device)
        src, hops = torch.empty(self.sim.N, **z), torch.empty(self.sim.N, **z)
        _ns._check(_lib().navsim_rp_attach_outputs(self.h, _ptr(src), _ptr(hops),
                                                   self._stream()))
        return src, hops

    def forward(self, x_bits: torch.Tensor) -> torch.Tensor:
        n = x_bits.shape[0]
        assert x_bits.dtype == torch.int16 and x_bits.shape[1] == self.d0
        y = torch.empty(n, 5, dtype=torch.float32, device=self.device)
        _ns._check(_lib().navsim_rp_forward(self.h, n, _ptr(x_bits), _ptr(y), self._stream()))
        return y

    def loss_grad(self, x_bits, target):
        n = x_bits.shape[0]
        rows = torch.empty(n, dtype=torch.float32, device=self.device)
        g = torch.empty(self.count, dtype=torch.float32, device=self.device)
        _ns._check(_lib().navsim_rp_loss_grad(self.h, n, _ptr(x_bits), _ptr(target),
                                              _ptr(rows), _ptr(g), self._stream()))
        return rows, g

    def adamw(self, grad, lr: float, weight_decay: float):
        _ns._check(_lib().navsim_rp_adamw(self.h, _ptr(grad, torch.float32), float(lr),
                                          float(weight_decay), self._stream()))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.count, np.float32)
        _ns._check(_lib().navsim_rp_get_params(self.h, out.ctypes.data, self.count))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _ns._check(_lib().navsim_rp_set_params(self.h, p.ctypes.data, self.count))
