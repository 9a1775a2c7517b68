"""Per-map robot/sensor profiles in the oracle: a batch that mixes beam counts
and footprints must give, for the envs on each map, exactly what a batch run
entirely with that map's robot and sensor gives (profiles only choose which
robot of section 2.2 / appendix B an env carries)."""
import math

import numpy as np

import oracle
from workloads import configs
from workloads import maps as gm

PROFILES = [dict(num_beams=60, footprint=0, radius_m=0.18, length_m=0.0, width_m=0.0),
            dict(num_beams=240, footprint=1, radius_m=0.0, length_m=0.70, width_m=0.31),
            dict(num_beams=120, footprint=1, radius_m=0.0, length_m=0.80, width_m=0.41)]


def _setup(num_envs=45):
    occ = [gm.gen_rect_disc_map(21, w=60, h=44, res=0.05),
           gm.gen_rooms_map(22, w=90, h=70, res=0.05),
           gm.gen_rect_disc_map(23, w=40, h=80, res=0.05)]
    cfg = configs.make_config(num_envs=num_envs, num_beams=240, num_sectors=6,
                              fov_rad=2 * math.pi, max_range_m=4.0, dt_s=0.1, footprint=0,
                              radius_m=0.18, v_min=-0.5, v_max=0.5, w_min=-1.0, w_max=1.0)
    env_map = (np.arange(num_envs) % 3).astype(np.int32)
    return cfg, occ, [0.05] * 3, env_map


def test_mixed_batch_equals_per_profile_batches():
    cfg, occ, res, env_map = _setup()
    acts = configs.uniform_actions(6, cfg["num_envs"], seed=3)
    mixed = oracle.OracleSim(cfg, occ, res, env_map, profiles=PROFILES)
    mo, _ = mixed.reset()
    mouts = [mixed.step(a) for a in acts]
    assert sum(int(o["reset"].sum()) for o in mouts) > 0  # auto-resets are covered
    for k, q in enumerate(PROFILES):
        c = dict(cfg)
        c.update(num_beams=q["num_beams"], footprint=q["footprint"], radius_m=q["radius_m"],
                 length_m=q["length_m"], width_m=q["width_m"])
        one = oracle.OracleSim(c, occ, res, env_map)
        oo, _ = one.reset()
        rows = env_map == k
        assert np.array_equal(mo[rows], oo[rows])
        for t, a in enumerate(acts):
            o = one.step(a)
            for key in ("obs", "reward", "terminated", "truncated", "final_obs", "collision",
                        "goal", "reset", "fallback"):
                assert np.array_equal(mouts[t][key][rows], o[key][rows]), (k, t, key)
            K = q["num_beams"]
            for key in ("ranges", "hits", "grazing", "visits"):
                assert np.array_equal(mouts[t][key][rows, :K], o[key][rows]), (k, t, key)
                assert not mouts[t][key][rows, K:].any(), (k, t, key)


def test_footprint_profile_changes_collision_only_through_the_footprint():
    # the same pose next to a wall collides with the long rectangle and not
    # with the small disc: profile 1's free list must exclude cells that
    # profile 0's includes
    cfg, occ, res, env_map = _setup()
    mixed = oracle.OracleSim(cfg, occ, res, env_map, profiles=PROFILES)
    M = mixed.maps
    assert M.free_cnt[0] > 0 and M.free_cnt[1] > 0 and M.free_cnt[2] > 0
    same = oracle.OracleSim(dict(cfg, footprint=0, radius_m=0.18), occ, res, env_map)
    # rectangle circumradius 0.38 m > disc 0.18 m: fewer free cells on maps 1, 2
    assert M.free_cnt[1] < same.maps.free_cnt[1]
    assert M.free_cnt[2] < same.maps.free_cnt[2]
    assert M.free_cnt[0] == same.maps.free_cnt[0]
