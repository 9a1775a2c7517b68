"""CPU oracle for the batched bitmap navigation step.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg are the only code that may import this package.  The GPU
library never loads it, and it shares no code with the GPU library: the
arithmetic lives in ``navsim_oracle.c`` (plain scalar double precision C),
this module only marshals numpy arrays into it.

What each C function computes and which part of the paper it follows is
written beside it in ``navsim_oracle.c``.
"""
from __future__ import annotations

import concurrent.futures as _cf
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))

STATE_KEYS = ("x", "y", "th", "v", "w", "gx", "gy", "dprev", "t", "ep")
_STATE_DTYPES = dict(x=np.float32, y=np.float32, th=np.float32, v=np.float32, w=np.float32,
                     gx=np.float32, gy=np.float32, dprev=np.float32, t=np.int32, ep=np.uint32)


class OrcCfg(C.Structure):
    _fields_ = [
        ("num_envs", C.c_int32), ("num_beams", C.c_int32), ("num_sectors", C.c_int32),
        ("fov_rad", C.c_float), ("max_range_m", C.c_float), ("dt_s", C.c_float),
        ("horizon", C.c_int32),
        ("goal_radius_m", C.c_float), ("c_progress", C.c_float), ("r_success", C.c_float),
        ("r_collision", C.c_float),
        ("footprint", C.c_int32),
        ("radius_m", C.c_float), ("length_m", C.c_float), ("width_m", C.c_float),
        ("v_min", C.c_float), ("v_max", C.c_float), ("w_min", C.c_float), ("w_max", C.c_float),
        ("goal_min_dist_m", C.c_float),
        ("reset_max_tries", C.c_int32),
        ("seed", C.c_uint64),
        ("scan_mode", C.c_int32), ("march_step_m", C.c_float),
    ]


class OrcMaps(C.Structure):
    _fields_ = [
        ("num_maps", C.c_int32),
        ("w", C.POINTER(C.c_int32)), ("h", C.POINTER(C.c_int32)), ("res", C.POINTER(C.c_float)),
        ("off", C.POINTER(C.c_int64)), ("occ", C.POINTER(C.c_uint8)),
        ("free_off", C.POINTER(C.c_int64)), ("free_cnt", C.POINTER(C.c_int32)),
        ("free_cells", C.POINTER(C.c_int32)),
        ("prof_beams", C.POINTER(C.c_int32)), ("prof_footprint", C.POINTER(C.c_int32)),
        ("prof_radius", C.POINTER(C.c_float)), ("prof_length", C.POINTER(C.c_float)),
        ("prof_width", C.POINTER(C.c_float)),
    ]


class OrcState(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_float)) for k in ("x", "y", "th", "v", "w", "gx", "gy", "dprev")] + [
        ("t", C.POINTER(C.c_int32)), ("ep", C.POINTER(C.c_uint32)), ("map", C.POINTER(C.c_int32)),
    ]


class OrcOut(C.Structure):
    _fields_ = [
        ("obs", C.POINTER(C.c_float)), ("reward", C.POINTER(C.c_float)),
        ("terminated", C.POINTER(C.c_uint8)), ("truncated", C.POINTER(C.c_uint8)),
        ("final_obs", C.POINTER(C.c_float)),
        ("ranges", C.POINTER(C.c_float)), ("hits", C.POINTER(C.c_int32)),
        ("grazing", C.POINTER(C.c_uint8)), ("visits", C.POINTER(C.c_int32)),
        ("collision", C.POINTER(C.c_uint8)), ("goal", C.POINTER(C.c_uint8)),
        ("reset", C.POINTER(C.c_uint8)), ("fallback", C.POINTER(C.c_uint8)),
    ]


class OrcRay(C.Structure):
    _fields_ = [("range", C.c_double), ("perp", C.c_double), ("t_end", C.c_double),
                ("hit", C.c_int32), ("visits", C.c_int32), ("grazing", C.c_int32),
                ("pad", C.c_int32)]


_LIB = None


def lib():
    """Load liborc.so, compiling it first when it is not there."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(_HERE, "liborc.so")
    if not os.path.exists(path):
        _build.build()
    L = C.CDLL(path)
    P = C.POINTER
    L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
    L.orc_occupied.argtypes = [P(OrcMaps), C.c_int, C.c_int64, C.c_int64]
    L.orc_disc_hits.argtypes = [P(OrcMaps), C.c_int, C.c_double, C.c_double, C.c_double]
    L.orc_rect_hits.argtypes = [P(OrcMaps), C.c_int, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_double]
    L.orc_footprint_hits.argtypes = [P(OrcMaps), C.c_int, P(OrcCfg), C.c_double, C.c_double,
                                     C.c_double]
    L.orc_circumradius.argtypes = [P(OrcCfg)]
    L.orc_circumradius.restype = C.c_double
    L.orc_free_list.argtypes = [P(OrcMaps), C.c_int, C.c_double, P(C.c_int32)]
    L.orc_free_list.restype = C.c_int64
    L.orc_cast.argtypes = [P(OrcMaps), C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                           C.c_double, C.c_double, P(OrcRay)]
    L.orc_march.argtypes = [P(OrcMaps), C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                            C.c_double, C.c_double, P(C.c_double), P(C.c_int32), P(C.c_int32),
                            P(C.c_double)]
    L.orc_cfg_for_map.argtypes = [P(OrcCfg), P(OrcMaps), C.c_int, P(OrcCfg)]
    L.orc_reset_to.argtypes = [P(OrcCfg), P(OrcMaps), P(OrcState), P(C.c_uint8), P(C.c_float),
                               P(C.c_float), C.c_int64, C.c_int64]
    L.orc_rollout_actions.argtypes = [P(OrcCfg), C.c_uint64, C.c_int64, C.c_int64, P(C.c_float)]
    L.orc_beam_angle.argtypes = [P(OrcCfg), C.c_int]
    L.orc_beam_angle.restype = C.c_double
    L.orc_scan.argtypes = [P(OrcMaps), C.c_int, P(OrcCfg), C.c_double, C.c_double, C.c_double,
                           P(C.c_float), P(C.c_int32), P(C.c_uint8), P(C.c_int32)]
    L.orc_reset.argtypes = [P(OrcCfg), P(OrcMaps), P(OrcState), P(C.c_uint8), P(C.c_float),
                            P(C.c_uint8), C.c_int64, C.c_int64]
    L.orc_step.argtypes = [P(OrcCfg), P(OrcMaps), P(OrcState), P(C.c_float), P(OrcOut),
                           C.c_int64, C.c_int64]
    L.orc_step_defer.argtypes = [P(OrcCfg), P(OrcMaps), P(OrcState), P(C.c_float), P(OrcOut),
                                 P(C.c_int32), C.c_int64, C.c_int64]
    _LIB = L
    return L


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


def philox4x32_10(ctr, key) -> tuple:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(int(v) for v in o)


_CFG_DEFAULTS = dict(scan_mode=0, march_step_m=0.03)


def make_cfg(cfg: dict) -> OrcCfg:
    """scan_mode (0 traversal, 1 fixed-step march) and march_step_m default to
    0 and 0.03 m (table 7) when the dict does not give them."""
    c = OrcCfg()
    for name, _ in OrcCfg._fields_:
        setattr(c, name, cfg.get(name, _CFG_DEFAULTS.get(name)) if name in _CFG_DEFAULTS
                else cfg[name])
    return c


class OracleMaps:
    """Maps concatenated for the oracle, with the free-cell lists it builds and
    optional per-map robot/sensor profiles (dicts with num_beams, footprint,
    radius_m, length_m, width_m)."""

    def __init__(self, maps, res, circumradius: float | None = None, profiles=None):
        self.maps = [np.ascontiguousarray(m, dtype=np.uint8) for m in maps]
        n = len(self.maps)
        self.w = np.array([m.shape[1] for m in self.maps], dtype=np.int32)
        self.h = np.array([m.shape[0] for m in self.maps], dtype=np.int32)
        self.res = np.array(res, dtype=np.float32)
        sizes = np.array([m.size for m in self.maps], dtype=np.int64)
        self.off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        self.occ = np.concatenate([m.ravel() for m in self.maps]) if n else np.zeros(0, np.uint8)
        self.free_off = np.zeros(n, dtype=np.int64)
        self.free_cnt = np.zeros(n, dtype=np.int32)
        self.free_cells = np.zeros(1, dtype=np.int32)
        self.profiles = profiles
        if profiles is not None:
            self.p_beams = np.array([q["num_beams"] for q in profiles], np.int32)
            self.p_fp = np.array([q["footprint"] for q in profiles], np.int32)
            self.p_rad = np.array([q.get("radius_m", 0.0) for q in profiles], np.float32)
            self.p_len = np.array([q.get("length_m", 0.0) for q in profiles], np.float32)
            self.p_wid = np.array([q.get("width_m", 0.0) for q in profiles], np.float32)
        self._mk()
        if circumradius is not None:
            self.build_free_lists(circumradius)

    def _mk(self):
        pr = self.profiles is not None
        self.struct = OrcMaps(
            int(len(self.maps)), _ptr(self.w, C.c_int32), _ptr(self.h, C.c_int32),
            _ptr(self.res, C.c_float), _ptr(self.off, C.c_int64), _ptr(self.occ, C.c_uint8),
            _ptr(self.free_off, C.c_int64), _ptr(self.free_cnt, C.c_int32),
            _ptr(self.free_cells, C.c_int32),
            _ptr(self.p_beams, C.c_int32) if pr else None, _ptr(self.p_fp, C.c_int32) if pr else None,
            _ptr(self.p_rad, C.c_float) if pr else None, _ptr(self.p_len, C.c_float) if pr else None,
            _ptr(self.p_wid, C.c_float) if pr else None)

    def build_free_lists(self, rc):
        """rc: one circumradius for every map, or a list with one per map."""
        L = lib()
        lists = []
        rcs = list(rc) if np.ndim(rc) else [rc] * len(self.maps)
        for k in range(len(self.maps)):
            buf = np.zeros(int(self.w[k]) * int(self.h[k]), dtype=np.int32)
            cnt = L.orc_free_list(C.byref(self.struct), k, float(rcs[k]), _ptr(buf, C.c_int32))
            lists.append(buf[:cnt])
        self.free_cnt = np.array([len(x) for x in lists], dtype=np.int32)
        self.free_off = np.concatenate([[0], np.cumsum(self.free_cnt)[:-1]]).astype(np.int64)
        self.free_cells = (np.concatenate(lists) if lists else np.zeros(0, np.int32)).astype(np.int32)
        if self.free_cells.size == 0:
            self.free_cells = np.zeros(1, dtype=np.int32)
        self._mk()

    # --- single-query helpers (tests) ---
    def occupied(self, k, i, j) -> bool:
        return bool(lib().orc_occupied(C.byref(self.struct), k, int(i), int(j)))

    def disc_hits(self, k, x, y, r) -> bool:
        return bool(lib().orc_disc_hits(C.byref(self.struct), k, float(x), float(y), float(r)))

    def rect_hits(self, k, x, y, th, L_, B_) -> bool:
        return bool(lib().orc_rect_hits(C.byref(self.struct), k, float(x), float(y), float(th),
                                         float(L_), float(B_)))

    def cast(self, k, ox, oy, dx, dy, rmax, eps=1e-6) -> OrcRay:
        r = OrcRay()
        lib().orc_cast(C.byref(self.struct), k, float(ox), float(oy), float(dx), float(dy),
                       float(rmax), float(eps), C.byref(r))
        return r

    def march(self, k, ox, oy, dx, dy, rmax, h):
        rg = C.c_double()
        hit = C.c_int32()
        ns = C.c_int32()
        nr = C.c_double()
        lib().orc_march(C.byref(self.struct), k, float(ox), float(oy), float(dx), float(dy),
                        float(rmax), float(h), C.byref(rg), C.byref(hit), C.byref(ns), C.byref(nr))
        return rg.value, hit.value


class OracleSim:
    """Batched simulator state on the CPU, stepped by the C oracle."""

    def __init__(self, cfg: dict, maps, res, env_map, profiles=None):
        self.cfg_dict = dict(cfg)
        self.cfg = make_cfg(cfg)
        self.N = int(cfg["num_envs"])
        self.K = int(cfg["num_beams"])  # largest beam count: stride of per-ray outputs
        self.m = int(cfg["num_sectors"])
        L = lib()
        self.maps = OracleMaps(maps, res, profiles=profiles)
        rcs = []
        for k in range(len(maps)):
            mc = OrcCfg()
            L.orc_cfg_for_map(C.byref(self.cfg), C.byref(self.maps.struct), k, C.byref(mc))
            rcs.append(L.orc_circumradius(C.byref(mc)))
        self.maps.build_free_lists(rcs)
        self.env_map = np.ascontiguousarray(env_map, dtype=np.int32)
        self.state = {k: np.zeros(self.N, dtype=_STATE_DTYPES[k]) for k in STATE_KEYS}
        self._mk_state()

    def _mk_state(self):
        s = self.state
        self.st = OrcState(*[_ptr(s[k], C.c_float) for k in ("x", "y", "th", "v", "w", "gx", "gy",
                                                             "dprev")],
                           _ptr(s["t"], C.c_int32), _ptr(s["ep"], C.c_uint32),
                           _ptr(self.env_map, C.c_int32))

    def get_state(self) -> dict:
        return {k: v.copy() for k, v in self.state.items()}

    def set_state(self, st: dict):
        for k in STATE_KEYS:
            self.state[k][:] = np.asarray(st[k]).astype(_STATE_DTYPES[k])

    def _slices(self, threads):
        threads = max(1, int(threads))
        edges = np.linspace(0, self.N, threads + 1).astype(np.int64)
        return [(int(a), int(b)) for a, b in zip(edges[:-1], edges[1:]) if b > a]

    def reset(self, mask=None, threads: int = 1):
        obs = np.zeros((self.N, self.m + 4), dtype=np.float32)
        fb = np.zeros(self.N, dtype=np.uint8)
        mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        L = lib()

        def run(sl):
            L.orc_reset(C.byref(self.cfg), C.byref(self.maps.struct), C.byref(self.st),
                        _ptr(mk, C.c_uint8), _ptr(obs, C.c_float), _ptr(fb, C.c_uint8), sl[0],
                        sl[1])
        self._run(run, threads)
        return obs, fb

    def _run(self, fn, threads):
        sl = self._slices(threads)
        if len(sl) == 1:
            fn(sl[0])
            return
        with _cf.ThreadPoolExecutor(len(sl)) as ex:
            list(ex.map(fn, sl))

    def step(self, act, debug: bool = True, threads: int = 1, defer_bin=None) -> dict:
        """One step of every env; with defer_bin [N] (int32), envs that end
        with defer_bin[e] >= 0 are not reset (orc_step_defer)."""
        N, K, m = self.N, self.K, self.m
        act = np.ascontiguousarray(act, dtype=np.float32).reshape(N, 2)
        o = dict(obs=np.zeros((N, m + 4), np.float32), reward=np.zeros(N, np.float32),
                 terminated=np.zeros(N, np.uint8), truncated=np.zeros(N, np.uint8),
                 final_obs=np.zeros((N, m + 4), np.float32), collision=np.zeros(N, np.uint8),
                 goal=np.zeros(N, np.uint8), reset=np.zeros(N, np.uint8),
                 fallback=np.zeros(N, np.uint8))
        if debug:
            o.update(ranges=np.zeros((N, K), np.float32), hits=np.zeros((N, K), np.int32),
                     grazing=np.zeros((N, K), np.uint8), visits=np.zeros((N, K), np.int32))
        out = OrcOut(_ptr(o["obs"], C.c_float), _ptr(o["reward"], C.c_float),
                     _ptr(o["terminated"], C.c_uint8), _ptr(o["truncated"], C.c_uint8),
                     _ptr(o["final_obs"], C.c_float),
                     _ptr(o.get("ranges"), C.c_float), _ptr(o.get("hits"), C.c_int32),
                     _ptr(o.get("grazing"), C.c_uint8), _ptr(o.get("visits"), C.c_int32),
                     _ptr(o["collision"], C.c_uint8), _ptr(o["goal"], C.c_uint8),
                     _ptr(o["reset"], C.c_uint8), _ptr(o["fallback"], C.c_uint8))
        L = lib()

        db = None if defer_bin is None else np.ascontiguousarray(defer_bin, dtype=np.int32)

        def run(sl):
            L.orc_step_defer(C.byref(self.cfg), C.byref(self.maps.struct), C.byref(self.st),
                             _ptr(act, C.c_float), C.byref(out), _ptr(db, C.c_int32), sl[0],
                             sl[1])
        self._run(run, threads)
        return o

    def reset_to(self, pose, mask=None) -> np.ndarray:
        """Reset masked envs to given poses [N, 5]; returns the obs rows (zeros
        for unmasked envs)."""
        obs = np.zeros((self.N, self.m + 4), dtype=np.float32)
        pz = np.ascontiguousarray(pose, dtype=np.float32)
        mk = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
        lib().orc_reset_to(C.byref(self.cfg), C.byref(self.maps.struct), C.byref(self.st),
                           _ptr(mk, C.c_uint8), _ptr(pz, C.c_float), _ptr(obs, C.c_float), 0,
                           self.N)
        return obs

    def rollout_actions(self, n: int) -> np.ndarray:
        """Normalised actions [N, 2] of rollout step n (Philox stream 4)."""
        a = np.zeros((self.N, 2), np.float32)
        lib().orc_rollout_actions(C.byref(self.cfg), int(n), 0, self.N, _ptr(a, C.c_float))
        return a

    def map_cfg(self, map_id) -> OrcCfg:
        mc = OrcCfg()
        lib().orc_cfg_for_map(C.byref(self.cfg), C.byref(self.maps.struct), int(map_id),
                              C.byref(mc))
        return mc

    def scan(self, map_id, x, y, th):
        mc = self.map_cfg(map_id)
        K = int(mc.num_beams)
        rg = np.zeros(K, np.float32)
        hit = np.zeros(K, np.int32)
        gr = np.zeros(K, np.uint8)
        vis = np.zeros(K, np.int32)
        lib().orc_scan(C.byref(self.maps.struct), int(map_id), C.byref(mc), float(x),
                       float(y), float(th), _ptr(rg, C.c_float), _ptr(hit, C.c_int32),
                       _ptr(gr, C.c_uint8), _ptr(vis, C.c_int32))
        return rg, hit, gr, vis

    def beam_angle(self, k) -> float:
        return lib().orc_beam_angle(C.byref(self.cfg), int(k))

    def collides(self, map_id, x, y, th) -> bool:
        mc = self.map_cfg(map_id)
        return bool(lib().orc_footprint_hits(C.byref(self.maps.struct), int(map_id),
                                             C.byref(mc), float(x), float(y), float(th)))
