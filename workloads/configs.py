"""Workload presets: simulator parameters, maps, env-to-map assignment and
seeded action streams.

Only input data and parameter values live here.  The simulator parameters of
the paper's two robots come from appendix B (table 7 shared sensor/episode
values, table 8 TurtleBot2, table 9 Go2).  The numbered workloads are the
synthetic configurations this project measures on; their maps are drawn by
``workloads.maps``.
"""
from __future__ import annotations

import math

import numpy as np

from . import maps as _maps

FOOTPRINT_DISC = 0
FOOTPRINT_RECT = 1

# Field order matches the C struct in include/navsim.h (the oracle keeps its
# own copy of the struct; this is only the list of parameter names).
CONFIG_FIELDS = (
    "num_envs", "num_beams", "num_sectors", "fov_rad", "max_range_m", "dt_s",
    "horizon", "goal_radius_m", "c_progress", "r_success", "r_collision",
    "footprint", "radius_m", "length_m", "width_m", "v_min", "v_max", "w_min",
    "w_max", "goal_min_dist_m", "reset_max_tries", "seed",
)

_COMMON = dict(
    horizon=200,          # table 7: episode horizon 200 steps
    goal_radius_m=0.2,    # table 7: goal-reach threshold
    c_progress=2.0,       # table 7 / eq. 3: progress reward 2 (d_old - d_new)
    r_success=10.0,       # table 7: goal-reach reward
    r_collision=-10.0,    # table 7: collision penalty
    goal_min_dist_m=1.0,
    reset_max_tries=64,
    length_m=0.0,
    width_m=0.0,
    radius_m=0.0,
    seed=0x5EED,
)


def make_config(**kw) -> dict:
    cfg = dict(_COMMON)
    cfg.update(kw)
    missing = [f for f in CONFIG_FIELDS if f not in cfg]
    if missing:
        raise KeyError(f"config is missing {missing}")
    return cfg


# --- the paper's robots (appendix B) ---------------------------------------
def turtlebot2(num_envs: int = 1024) -> dict:
    """Table 7 + table 8: disc r = 0.2 m, 270 deg FOV, 1080 beams -> 30 sectors,
    r_max 20 m, dt 0.1 s, action bounds v in [0, 0.5], w in [-pi/4, pi/4]."""
    return make_config(num_envs=num_envs, num_beams=1080, num_sectors=30,
                       fov_rad=math.radians(270.0), max_range_m=20.0, dt_s=0.1,
                       footprint=FOOTPRINT_DISC, radius_m=0.2,
                       v_min=0.0, v_max=0.5, w_min=-math.pi / 4, w_max=math.pi / 4)


def go2(num_envs: int = 1024) -> dict:
    """Table 7 + table 9: 0.80 x 0.41 m rectangle, 360 deg FOV, 1080 beams,
    r_max 20 m, v in [0, 0.5], w in [-pi/4, pi/4]."""
    return make_config(num_envs=num_envs, num_beams=1080, num_sectors=30,
                       fov_rad=2 * math.pi, max_range_m=20.0, dt_s=0.1,
                       footprint=FOOTPRINT_RECT, length_m=0.80, width_m=0.41,
                       v_min=0.0, v_max=0.5, w_min=-math.pi / 4, w_max=math.pi / 4)


# --- measured workloads ------------------------------------------------------
WORKLOADS = {
    # 16 envs, one 64x64 map at 0.1 m, rectangles ~10 %, disc r 0.18, 36 beams
    # over 360 deg, r_max 3.5 m, dt 0.1, 200 steps with auto-reset.
    "c1": dict(cfg=dict(num_envs=16, num_beams=36, num_sectors=36, fov_rad=2 * math.pi,
                        max_range_m=3.5, dt_s=0.1, footprint=FOOTPRINT_DISC, radius_m=0.18,
                        v_min=0.0, v_max=0.5, w_min=-1.0, w_max=1.0),
               maps=dict(kind="rect", count=1, w=64, h=64, res=0.1), steps=200,
               name="16 envs, 1 map 64x64 @0.1 m, disc r 0.18 m, 36 beams, r_max 3.5 m"),
    # 4096 envs over 16 maps 128x128 at 0.05 m (rectangles + discs, 15 %),
    # disc r 0.18, 360 beams -> 30 sectors, r_max 6 m, dt 0.1, 1000 steps.
    "c2": dict(cfg=dict(num_envs=4096, num_beams=360, num_sectors=30, fov_rad=2 * math.pi,
                        max_range_m=6.0, dt_s=0.1, footprint=FOOTPRINT_DISC, radius_m=0.18,
                        v_min=0.0, v_max=0.5, w_min=-1.0, w_max=1.0),
               maps=dict(kind="rect_disc", count=16, w=128, h=128, res=0.05), steps=1000,
               name="4096 envs, 16 maps 128x128 @0.05 m, disc r 0.18 m, 360 beams, r_max 6 m"),
    # 16384 envs over 64 maps 256x256 (rooms + clutter), 0.70 x 0.31 m
    # rectangle, 720 beams -> 30 sectors, r_max 8 m, dt 0.05, reverse allowed.
    "c3": dict(cfg=dict(num_envs=16384, num_beams=720, num_sectors=30, fov_rad=2 * math.pi,
                        max_range_m=8.0, dt_s=0.05, footprint=FOOTPRINT_RECT,
                        length_m=0.70, width_m=0.31,
                        v_min=-0.5, v_max=0.5, w_min=-1.0, w_max=1.0),
               maps=dict(kind="rooms", count=64, w=256, h=256, res=0.05), steps=2000,
               name="16384 envs, 64 maps 256x256 @0.05 m, rect 0.70x0.31 m, 720 beams, r_max 8 m"),
    # 32768 envs over 128 maps with W, H each U{96..512} at 0.05 m (rectangle+disc
    # and rooms generators alternating), per-map beam count from
    # {180, 360, 720, 1080} and disc (r 0.18) or rectangle (0.70 x 0.31 m)
    # footprint, m = 30, r_max 8 m, dt 0.05, reverse allowed.
    "c4": dict(cfg=dict(num_envs=32768, num_beams=1080, num_sectors=30, fov_rad=2 * math.pi,
                        max_range_m=8.0, dt_s=0.05, footprint=FOOTPRINT_DISC, radius_m=0.18,
                        v_min=-0.5, v_max=0.5, w_min=-1.0, w_max=1.0),
               maps=dict(kind="uneven", count=128, side_lo=96, side_hi=512, res=0.05,
                         seed=404),
               profiles=dict(seed=405, beams=(180, 360, 720, 1080),
                             disc=dict(footprint=FOOTPRINT_DISC, radius_m=0.18),
                             rect=dict(footprint=FOOTPRINT_RECT, length_m=0.70, width_m=0.31)),
               steps=64,
               name="32768 envs, 128 maps U{96..512}^2 @0.05 m, per-map K in "
                    "{180,360,720,1080} and disc/rect footprint, r_max 8 m"),
    # 65536 envs over 64 maps 256x256 at 0.05 m (rooms and corridors with disc
    # clutter), disc r 0.18 m, 360 beams -> 30 sectors, r_max 6 m; resets at a
    # requested geodesic difficulty (8 bins over 1-12 m) by the learned proposal.
    "c5": dict(cfg=dict(num_envs=65536, num_beams=360, num_sectors=30, fov_rad=2 * math.pi,
                        max_range_m=6.0, dt_s=0.1, footprint=FOOTPRINT_DISC, radius_m=0.18,
                        v_min=0.0, v_max=0.5, w_min=-1.0, w_max=1.0),
               maps=dict(kind="rooms", count=64, w=256, h=256, res=0.05, seed0=3000),
               proposer=dict(num_bins=8, d_lo_m=1.0, d_hi_m=12.0, noise_dim=16, hidden=256,
                             hidden_layers=3, leaky_slope=0.01, seed=0xC0FFEE),
               steps=200,
               name="65536 envs, 64 rooms maps 256x256 @0.05 m, disc r 0.18 m, 360 beams, "
                    "difficulty resets (8 bins, 1-12 m)"),
}


def build_profiles(spec: dict, count: int) -> list[dict]:
    """Per-map robot/sensor profiles: beam count drawn uniformly from
    spec['beams'], footprint disc or rectangle with probability 1/2."""
    rng = np.random.default_rng(spec["seed"])
    out = []
    for _ in range(count):
        k = int(rng.choice(np.asarray(spec["beams"])))
        fp = dict(spec["rect"] if rng.integers(0, 2) else spec["disc"])
        q = dict(num_beams=k, radius_m=0.0, length_m=0.0, width_m=0.0)
        q.update(fp)
        out.append(q)
    return out


def build_maps(spec: dict) -> tuple[list[np.ndarray], list[float]]:
    kind, count = spec["kind"], spec["count"]
    res = spec["res"]
    if kind == "uneven":
        occ = _maps.gen_uneven_maps(spec["seed"], count, side_lo=spec["side_lo"],
                                    side_hi=spec["side_hi"], res=res)
        return occ, [res] * count
    out = []
    for k in range(count):
        seed = spec.get("seed0", 1000) + k
        if kind == "rect":
            out.append(_maps.gen_rect_map(seed, w=spec["w"], h=spec["h"]))
        elif kind == "rect_disc":
            out.append(_maps.gen_rect_disc_map(seed, w=spec["w"], h=spec["h"], res=res))
        elif kind == "rooms":
            out.append(_maps.gen_rooms_map(seed, w=spec["w"], h=spec["h"], res=res))
        else:
            raise ValueError(kind)
    return out, [res] * count


def contiguous_env_map(num_envs: int, num_maps: int) -> np.ndarray:
    """env e uses map floor(e * M / N): contiguous blocks of envs per map."""
    e = np.arange(num_envs, dtype=np.int64)
    return ((e * num_maps) // num_envs).astype(np.int32)


def uniform_actions(num_steps: int, num_envs: int, seed: int = 42) -> np.ndarray:
    """Normalised actions uniform on [-1, 1]^2, shape [steps, envs, 2], float32."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(num_steps, num_envs, 2)).astype(np.float32)


def build_workload(name: str, num_envs: int | None = None) -> dict:
    """Return cfg, maps, res, env_map for a named workload (optionally with a
    different env count on the same maps)."""
    spec = WORKLOADS[name]
    cfg = make_config(**spec["cfg"])
    if num_envs is not None:
        cfg["num_envs"] = int(num_envs)
    occ, res = build_maps(spec["maps"])
    env_map = contiguous_env_map(cfg["num_envs"], len(occ))
    profiles = build_profiles(spec["profiles"], len(occ)) if "profiles" in spec else None
    return dict(cfg=cfg, maps=occ, res=res, env_map=env_map, steps=spec["steps"],
                name=spec["name"], profiles=profiles, proposer=spec.get("proposer"))
