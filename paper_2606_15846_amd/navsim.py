"""Python binding of libnavsim.so (the C ABI in include/navsim.h).

Argument marshalling only: every step of the simulation runs in the HIP
library.  Device buffers are torch tensors on the simulator's device; the
calls enqueue on the current torch stream of that device unless a stream is
given.  If the library is not built, loading fails loudly: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnavsim.so")

NAVSIM_ABI_VERSION = 1
NAVSIM_DISC, NAVSIM_RECT = 0, 1
NAVSIM_KERNEL_FUSED, NAVSIM_KERNEL_PLAIN = 0, 1
NAVSIM_ROLLOUT_GRAPH = 1
NAVSIM_SCAN_TRAVERSAL, NAVSIM_SCAN_MARCH = 0, 1
STATUS = {0: "NAVSIM_OK", -1: "NAVSIM_E_INVALID_ARG", -2: "NAVSIM_E_BAD_HANDLE",
          -3: "NAVSIM_E_STATE", -4: "NAVSIM_E_NO_FREE_SPACE", -5: "NAVSIM_E_OOM",
          -6: "NAVSIM_E_HIP", -7: "NAVSIM_E_UNSUPPORTED"}
EXPORTS = ("navsim_create", "navsim_load_maps", "navsim_load_maps_ex", "navsim_reset",
           "navsim_reset_to", "navsim_step",
           "navsim_step_plain", "navsim_step_debug", "navsim_rollout", "navsim_set_scan",
           "navsim_set_tuning",
           "navsim_get_tuning",
           "navsim_get_state", "navsim_set_state", "navsim_destroy", "navsim_last_error")
PROBE_EXPORTS = ("navsim_probe_lds_read",)  # include/navsim_probe.h
STATE_KEYS = ("x", "y", "th", "v", "w", "gx", "gy", "dprev", "t", "ep")
_STATE_DT = (np.float32,) * 8 + (np.int32, np.uint32)


class NavsimConfig(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("num_envs", C.c_int32), ("num_beams", C.c_int32),
        ("num_sectors", C.c_int32), ("fov_rad", C.c_float), ("max_range_m", C.c_float),
        ("dt_s", C.c_float), ("horizon", C.c_int32), ("goal_radius_m", C.c_float),
        ("c_progress", C.c_float), ("r_success", C.c_float), ("r_collision", C.c_float),
        ("footprint", C.c_int32), ("radius_m", C.c_float), ("length_m", C.c_float),
        ("width_m", C.c_float), ("v_min", C.c_float), ("v_max", C.c_float),
        ("w_min", C.c_float), ("w_max", C.c_float), ("goal_min_dist_m", C.c_float),
        ("reset_max_tries", C.c_int32), ("seed", C.c_uint64),
    ]


class NavsimDebug(C.Structure):
    _fields_ = [("ranges", C.c_void_p), ("hits", C.c_void_p), ("visits", C.c_void_p),
                ("collision", C.c_void_p), ("goal", C.c_void_p), ("reset", C.c_void_p),
                ("fallback", C.c_void_p)]


class NavsimMapProfile(C.Structure):
    _fields_ = [("num_beams", C.c_int32), ("footprint", C.c_int32), ("radius_m", C.c_float),
                ("length_m", C.c_float), ("width_m", C.c_float)]


class NavsimTuning(C.Structure):
    _fields_ = [("tile_envs", C.c_int32), ("refill_at", C.c_int32), ("groups", C.c_int32),
                ("ray_slots", C.c_int32), ("walk", C.c_int32), ("persist", C.c_int32),
                ("threads", C.c_int32), ("balance", C.c_int32)]


class NavsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_LIB = None


def load_library(path: str = LIB_PATH):
    """Load libnavsim.so (built in-tree by __graft_entry__.build())."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(path)
    vp, i32 = C.c_void_p, C.c_int32
    L.navsim_create.argtypes = [C.POINTER(NavsimConfig), C.c_int, C.POINTER(vp)]
    L.navsim_load_maps.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.navsim_load_maps_ex.argtypes = [vp, i32, vp, vp, vp, vp, vp, C.POINTER(NavsimMapProfile)]
    L.navsim_reset.argtypes = [vp, vp, vp, vp]
    L.navsim_reset_to.argtypes = [vp, vp, vp, vp, vp]
    L.navsim_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.navsim_step_plain.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.navsim_step_debug.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(NavsimDebug), i32, vp]
    L.navsim_rollout.argtypes = [vp, i32, C.c_uint64, vp, vp, vp, vp, vp, vp, i32, i32, vp]
    L.navsim_set_scan.argtypes = [vp, i32, C.c_float]
    L.navsim_set_tuning.argtypes = [vp, C.POINTER(NavsimTuning)]
    L.navsim_get_tuning.argtypes = [vp, C.POINTER(NavsimTuning)]
    L.navsim_get_state.argtypes = [vp, vp, C.c_size_t, vp]
    L.navsim_set_state.argtypes = [vp, vp, C.c_size_t, vp]
    L.navsim_destroy.argtypes = [vp]
    L.navsim_last_error.restype = C.c_char_p
    L.navsim_probe_lds_read.argtypes = [C.c_int, i32, i32, i32, i32, vp,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]
    for name in EXPORTS + PROBE_EXPORTS:
        if name != "navsim_last_error":
            getattr(L, name).restype = C.c_int
    _LIB = L
    return L


def navsim_probe_lds_read(hip_device: int, threads: int, blocks: int, iters: int,
                          launches: int, want_words: bool = False):
    """LDS read bandwidth (include/navsim_probe.h): returns (ms per launch,
    bytes per launch, the stored words of the last launch or None)."""
    out = np.zeros(blocks * threads, np.uint32) if want_words else None
    ms, nb = C.c_double(), C.c_double()
    _check(load_library().navsim_probe_lds_read(
        int(hip_device), int(threads), int(blocks), int(iters), int(launches),
        None if out is None else out.ctypes.data_as(C.c_void_p), C.byref(ms), C.byref(nb)))
    return ms.value, nb.value, out


def navsim_last_error() -> str:
    return load_library().navsim_last_error().decode()


def _check(status: int):
    if status != 0:
        raise NavsimError(status, navsim_last_error())


def make_config(cfg: dict) -> NavsimConfig:
    c = NavsimConfig()
    c.abi_version = NAVSIM_ABI_VERSION
    for name, _ in NavsimConfig._fields_[1:]:
        setattr(c, name, cfg[name])
    return c


def _dev_ptr(t, dtype, shape, device, name, optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or t.device != device:
        raise ValueError(f"{name} must be a tensor on {device}")
    if t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return C.c_void_p(s.cuda_stream)


def navsim_create(cfg: dict, hip_device: int = 0):
    h = C.c_void_p()
    c = make_config(cfg)
    _check(load_library().navsim_create(C.byref(c), int(hip_device), C.byref(h)))
    return h


def _map_arrays(maps, res, env_map):
    maps = [np.ascontiguousarray(m, dtype=np.uint8) for m in maps]
    w = np.array([m.shape[1] for m in maps], np.int32)
    hh = np.array([m.shape[0] for m in maps], np.int32)
    r = np.asarray(res, np.float32)
    occ = np.ascontiguousarray(np.concatenate([m.ravel() for m in maps]))
    em = np.ascontiguousarray(env_map, dtype=np.int32)
    return len(maps), w, hh, r, occ, em


def navsim_load_maps(h, maps, res, env_map):
    n, w, hh, r, occ, em = _map_arrays(maps, res, env_map)
    _check(load_library().navsim_load_maps(h, n, w.ctypes.data, hh.ctypes.data, r.ctypes.data,
                                           occ.ctypes.data, em.ctypes.data))


def navsim_load_maps_ex(h, maps, res, env_map, profiles=None):
    """profiles: None, or one dict per map with num_beams, footprint and the
    footprint's sizes (radius_m, or length_m and width_m)."""
    n, w, hh, r, occ, em = _map_arrays(maps, res, env_map)
    arr = None
    if profiles is not None:
        if len(profiles) != n:
            raise ValueError(f"{len(profiles)} profiles for {n} maps")
        arr = (NavsimMapProfile * n)()
        for k, q in enumerate(profiles):
            arr[k] = NavsimMapProfile(int(q["num_beams"]), int(q["footprint"]),
                                      float(q.get("radius_m", 0.0)), float(q.get("length_m", 0.0)),
                                      float(q.get("width_m", 0.0)))
    _check(load_library().navsim_load_maps_ex(h, n, w.ctypes.data, hh.ctypes.data, r.ctypes.data,
                                              occ.ctypes.data, em.ctypes.data, arr))


def navsim_reset(h, mask, obs, stream=None):
    dev = obs.device
    _check(load_library().navsim_reset(
        h, None if mask is None else C.c_void_p(mask.data_ptr()), C.c_void_p(obs.data_ptr()),
        _stream_ptr(stream, dev)))


def navsim_step(h, act, obs, reward, terminated, truncated, final_obs=None, stream=None):
    _check(load_library().navsim_step(
        h, C.c_void_p(act.data_ptr()), C.c_void_p(obs.data_ptr()), C.c_void_p(reward.data_ptr()),
        C.c_void_p(terminated.data_ptr()), C.c_void_p(truncated.data_ptr()),
        None if final_obs is None else C.c_void_p(final_obs.data_ptr()),
        _stream_ptr(stream, obs.device)))


def navsim_step_plain(h, act, obs, reward, terminated, truncated, final_obs=None, stream=None):
    _check(load_library().navsim_step_plain(
        h, C.c_void_p(act.data_ptr()), C.c_void_p(obs.data_ptr()), C.c_void_p(reward.data_ptr()),
        C.c_void_p(terminated.data_ptr()), C.c_void_p(truncated.data_ptr()),
        None if final_obs is None else C.c_void_p(final_obs.data_ptr()),
        _stream_ptr(stream, obs.device)))


def navsim_step_debug(h, act, obs, reward, terminated, truncated, final_obs, dbg: dict,
                      kernel: int = NAVSIM_KERNEL_FUSED, stream=None):
    d = NavsimDebug()
    for name, _ in NavsimDebug._fields_:
        t = dbg.get(name)
        setattr(d, name, None if t is None else t.data_ptr())
    _check(load_library().navsim_step_debug(
        h, C.c_void_p(act.data_ptr()), C.c_void_p(obs.data_ptr()), C.c_void_p(reward.data_ptr()),
        C.c_void_p(terminated.data_ptr()), C.c_void_p(truncated.data_ptr()),
        None if final_obs is None else C.c_void_p(final_obs.data_ptr()), C.byref(d), int(kernel),
        _stream_ptr(stream, obs.device)))


def navsim_rollout(h, steps: int, first_step: int, act, obs, reward, terminated, truncated,
                   final_obs=None, kernel: int = NAVSIM_KERNEL_FUSED, graph: bool = True,
                   stream=None):
    """Device tensors with a leading [steps] axis (act and final_obs may be None)."""
    dev = obs.device
    N, row = obs.shape[1], obs.shape[2]
    T = int(steps)
    args = (_dev_ptr(act, torch.float32, (T, N, 2), dev, "act", optional=True),
            _dev_ptr(obs, torch.float32, (T, N, row), dev, "obs"),
            _dev_ptr(reward, torch.float32, (T, N), dev, "reward"),
            _dev_ptr(terminated, torch.uint8, (T, N), dev, "terminated"),
            _dev_ptr(truncated, torch.uint8, (T, N), dev, "truncated"),
            _dev_ptr(final_obs, torch.float32, (T, N, row), dev, "final_obs", optional=True))
    _check(load_library().navsim_rollout(h, T, int(first_step), *args, int(kernel),
                                         NAVSIM_ROLLOUT_GRAPH if graph else 0,
                                         _stream_ptr(stream, dev)))


def navsim_set_tuning(h, tile_envs: int, refill_at: int, groups: int, ray_slots: int = 0,
                      walk: int = 3, persist: int = 0, threads: int = 256, balance: int = 0):
    t = NavsimTuning(int(tile_envs), int(refill_at), int(groups), int(ray_slots), int(walk),
                     int(persist), int(threads), int(balance))
    _check(load_library().navsim_set_tuning(h, C.byref(t)))


def navsim_get_tuning(h) -> dict:
    t = NavsimTuning()
    _check(load_library().navsim_get_tuning(h, C.byref(t)))
    return {"tile_envs": t.tile_envs, "refill_at": t.refill_at, "groups": t.groups,
            "ray_slots": t.ray_slots, "walk": t.walk, "persist": t.persist, "threads": t.threads,
            "balance": t.balance}


def navsim_get_state(h, num_envs: int, stream=None, device=None) -> dict:
    buf = np.zeros(10 * num_envs, np.uint32)
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    _check(load_library().navsim_get_state(h, buf.ctypes.data, buf.nbytes,
                                           _stream_ptr(stream, dev)))
    out = {}
    for i, (k, dt) in enumerate(zip(STATE_KEYS, _STATE_DT)):
        out[k] = buf[i * num_envs:(i + 1) * num_envs].view(dt).copy()
    return out


def navsim_set_state(h, state: dict, num_envs: int, stream=None, device=None):
    buf = np.zeros(10 * num_envs, np.uint32)
    for i, (k, dt) in enumerate(zip(STATE_KEYS, _STATE_DT)):
        buf[i * num_envs:(i + 1) * num_envs] = np.asarray(state[k]).astype(dt).view(np.uint32)
    dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
    _check(load_library().navsim_set_state(h, buf.ctypes.data, buf.nbytes,
                                           _stream_ptr(stream, dev)))


def navsim_destroy(h):
    _check(load_library().navsim_destroy(h))


class NavSim:
    """Gymnasium-style vector environment over one navsim handle (section
    2.2.4): step() returns obs, reward, terminated, truncated and the final
    observation of the envs that ended."""

    def __init__(self, cfg: dict, maps, res, env_map, device: int | str = 0, profiles=None):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.cfg = dict(cfg)
        self.N, self.K, self.m = int(cfg["num_envs"]), int(cfg["num_beams"]), int(cfg["num_sectors"])
        self.h = None
        self._proposers = weakref.WeakSet()  # reset proposers built on this handle
        self.h = navsim_create(cfg, self.device.index or 0)
        try:
            navsim_load_maps_ex(self.h, maps, res, env_map, profiles)
        except Exception:
            h, self.h = self.h, None
            navsim_destroy(h)
            raise
        z = dict(device=self.device)
        self.obs = torch.zeros(self.N, self.m + 4, dtype=torch.float32, **z)
        self.final_obs = torch.zeros(self.N, self.m + 4, dtype=torch.float32, **z)
        self.reward = torch.zeros(self.N, dtype=torch.float32, **z)
        self.terminated = torch.zeros(self.N, dtype=torch.uint8, **z)
        self.truncated = torch.zeros(self.N, dtype=torch.uint8, **z)

    def close(self):
        # proposers hold the handle: the library refuses to free it before them
        for rp in list(getattr(self, "_proposers", ())):
            rp.close()
        h, self.h = getattr(self, "h", None), None
        if h is not None:
            navsim_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_act(self, act):
        _dev_ptr(act, torch.float32, (self.N, 2), self.device, "act")

    def reset(self, mask=None):
        if mask is not None:
            _dev_ptr(mask, torch.uint8, (self.N,), self.device, "mask")
        navsim_reset(self.h, mask, self.obs)
        return self.obs

    def reset_to(self, pose, mask=None):
        """Reset the masked envs (all when mask is None) to the rows of pose
        (device float32 [N, 5]: x, y, heading, goal x, goal y)."""
        _dev_ptr(pose, torch.float32, (self.N, 5), self.device, "pose")
        if mask is not None:
            _dev_ptr(mask, torch.uint8, (self.N,), self.device, "mask")
        _check(load_library().navsim_reset_to(
            self.h, None if mask is None else C.c_void_p(mask.data_ptr()),
            C.c_void_p(pose.data_ptr()), C.c_void_p(self.obs.data_ptr()),
            _stream_ptr(None, self.device)))
        return self.obs

    def step(self, act, plain: bool = False):
        self._check_act(act)
        fn = navsim_step_plain if plain else navsim_step
        fn(self.h, act, self.obs, self.reward, self.terminated, self.truncated, self.final_obs)
        return self.obs, self.reward, self.terminated, self.truncated, {"final_obs": self.final_obs}

    def step_debug(self, act, kernel=NAVSIM_KERNEL_FUSED):
        self._check_act(act)
        z = dict(device=self.device)
        dbg = dict(ranges=torch.zeros(self.N, self.K, dtype=torch.float32, **z),
                   hits=torch.zeros(self.N, self.K, dtype=torch.int32, **z),
                   visits=torch.zeros(self.N, self.K, dtype=torch.int32, **z),
                   collision=torch.zeros(self.N, dtype=torch.uint8, **z),
                   goal=torch.zeros(self.N, dtype=torch.uint8, **z),
                   reset=torch.zeros(self.N, dtype=torch.uint8, **z),
                   fallback=torch.zeros(self.N, dtype=torch.uint8, **z))
        navsim_step_debug(self.h, act, self.obs, self.reward, self.terminated, self.truncated,
                          self.final_obs, dbg, kernel)
        return dbg

    def rollout_buffers(self, steps: int, final_obs: bool = True) -> dict:
        z = dict(device=self.device)
        T, N, row = int(steps), self.N, self.m + 4
        return dict(act=torch.zeros(T, N, 2, dtype=torch.float32, **z),
                    obs=torch.zeros(T, N, row, dtype=torch.float32, **z),
                    reward=torch.zeros(T, N, dtype=torch.float32, **z),
                    terminated=torch.zeros(T, N, dtype=torch.uint8, **z),
                    truncated=torch.zeros(T, N, dtype=torch.uint8, **z),
                    final_obs=torch.zeros(T, N, row, dtype=torch.float32, **z) if final_obs
                    else None)

    def rollout(self, steps: int, first_step: int, buffers: dict | None = None,
                kernel: int = NAVSIM_KERNEL_FUSED, graph: bool = True) -> dict:
        """`steps` steps under the device-drawn actions of steps first_step,
        first_step + 1, ...; returns the per-step buffers (reused when given)."""
        b = buffers if buffers is not None else self.rollout_buffers(steps)
        navsim_rollout(self.h, steps, first_step, b["act"], b["obs"], b["reward"],
                       b["terminated"], b["truncated"], b["final_obs"], kernel, graph)
        return b

    def set_scan(self, mode: int, step_m: float = 0.03):
        """NAVSIM_SCAN_TRAVERSAL (exact) or NAVSIM_SCAN_MARCH (fixed step)."""
        _check(load_library().navsim_set_scan(self.h, int(mode), float(step_m)))

    def set_tuning(self, tile_envs: int, refill_at: int, groups: int, ray_slots: int = 0,
                   walk: int = 3, persist: int = 0, threads: int = 256, balance: int = 0):
        navsim_set_tuning(self.h, tile_envs, refill_at, groups, ray_slots, walk, persist, threads,
                          balance)

    def get_tuning(self) -> dict:
        return navsim_get_tuning(self.h)

    def get_state(self) -> dict:
        return navsim_get_state(self.h, self.N, device=self.device)

    def set_state(self, state: dict):
        navsim_set_state(self.h, state, self.N, device=self.device)
