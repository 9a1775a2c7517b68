"""Pins for the oracle's whole step: action map and kinematics (section
2.2.3), goal features (eq. 1), reward (eq. 3), termination/truncation
(section 2.2.3, horizon from table 7), pooling (eq. 6), and sparse reset with
the final observation kept apart (section 2.2.3)."""
import math

import numpy as np
import pytest

import oracle
from tests.test_oracle_geometry import brute_disc, brute_rect
from workloads import configs


def f32(v):
    return float(np.float32(v))


def base_cfg(**kw):
    cfg = configs.make_config(num_envs=1, num_beams=36, num_sectors=36, fov_rad=2 * math.pi,
                              max_range_m=3.0, dt_s=0.1, footprint=0, radius_m=0.18,
                              v_min=0.0, v_max=0.5, w_min=-1.0, w_max=1.0)
    cfg.update(kw)
    return cfg


def open_map(n=200):
    return np.zeros((n, n), np.uint8)


def make(cfg, occ=None, res=0.05, n_envs=None):
    if n_envs is not None:
        cfg = dict(cfg, num_envs=n_envs)
    occ = open_map() if occ is None else occ
    return oracle.OracleSim(cfg, [occ], [res], np.zeros(cfg["num_envs"], np.int32))


def put(sim, e=0, **kw):
    st = sim.get_state()
    for k, v in kw.items():
        st[k][e] = v
    sim.set_state(st)


def test_action_map_closed_forms():
    sim = make(base_cfg(num_envs=5))
    put(sim, 0)
    for e in range(5):
        put(sim, e, x=5.0, y=5.0, gx=7.0, gy=5.0, dprev=2.0)
    act = np.array([[1, 1], [-1, -1], [0, 0], [np.nan, np.nan], [7, -9]], np.float32)
    o = sim.step(act)
    m = sim.m
    v, w = o["obs"][:, m + 2], o["obs"][:, m + 3]
    assert list(v) == [0.5, 0.0, 0.25, 0.25, 0.5]
    assert list(w) == [1.0, -1.0, 0.0, 0.0, -1.0]


def test_straight_line_and_turn_in_place():
    sim = make(base_cfg(num_envs=2))
    th0 = f32(0.3)
    put(sim, 0, x=3.0, y=3.0, th=th0, gx=9.0, gy=9.0, dprev=8.0)
    put(sim, 1, x=6.0, y=6.0, th=f32(3.1), gx=1.0, gy=9.0, dprev=8.0)
    act = np.array([[1.0, 0.0], [-1.0, 1.0]], np.float32)   # (v=0.5, w=0), (v=0, w=1)
    th_expect = 3.1
    for n in range(1, 30):
        sim.step(act)
        st = sim.get_state()
        # straight line: x_n = x_0 + n v dt cos th (float32 rounding per step)
        assert abs(st["x"][0] - (3.0 + n * 0.05 * math.cos(th0))) < 1e-5
        assert abs(st["y"][0] - (3.0 + n * 0.05 * math.sin(th0))) < 1e-5
        assert st["th"][0] == th0
        # turn in place: position unchanged, heading advances by w dt, wrapped
        assert st["x"][1] == 6.0 and st["y"][1] == 6.0
        th_expect += 0.1
        if th_expect >= math.pi:
            th_expect -= 2 * math.pi
        assert abs(st["th"][1] - th_expect) < 1e-5
        assert -math.pi - 1e-6 <= st["th"][1] <= math.pi + 1e-6


def test_euler_polygon_lies_on_circle():
    # Constant (v, w): each step is a chord of length v dt, turning by w dt, so
    # the visited points are vertices of a regular polygon of circumradius
    # v dt / (2 sin(w dt / 2)).
    cfg = base_cfg(num_envs=1, w_min=-0.8, w_max=0.8)
    sim = make(cfg)
    put(sim, 0, x=5.0, y=4.0, th=0.0, gx=9.5, gy=9.5, dprev=8.0)
    act = np.array([[1.0, 1.0]], np.float32)  # v = 0.5, w = 0.8
    pts = [(5.0, 4.0)]
    for _ in range(20):
        sim.step(act)
        st = sim.get_state()
        pts.append((float(st["x"][0]), float(st["y"][0])))
    rho = 0.5 * 0.1 / (2 * math.sin(0.8 * 0.1 / 2))
    # heading 0 at p0: the centre lies on the first chord's perpendicular
    # bisector, rho cos(a) to the left of its midpoint (a = half a turn step),
    # i.e. at p0 + rho (sin a, cos a)
    a = 0.8 * 0.1 / 2
    cx = 5.0 + rho * math.sin(a)
    cy = 4.0 + rho * math.cos(a)
    for (px, py) in pts:
        assert abs(math.hypot(px - cx, py - cy) - rho) < 2e-5


def test_goal_features_ahead_and_left():
    sim = make(base_cfg(num_envs=2))
    put(sim, 0, x=2.0, y=2.0, th=0.0, gx=4.5, gy=2.0, dprev=2.5)
    put(sim, 1, x=2.0, y=2.0, th=f32(math.pi / 2), gx=1.0, gy=2.0, dprev=1.0)
    o = sim.step(np.array([[-1.0, 0.0], [-1.0, 0.0]], np.float32))  # v = w = 0
    m = sim.m
    assert o["obs"][0, m] == 2.5 and o["obs"][0, m + 1] == 0.0
    assert o["obs"][1, m] == 1.0
    assert abs(o["obs"][1, m + 1] - math.pi / 2) < 1e-6   # goal is to the robot's left


def test_reward_and_flag_truth_table():
    occ = open_map()
    occ[:, 100] = 1                                       # wall face at x = 100 s
    s = f32(0.05)
    cfg = base_cfg(num_envs=5, horizon=200)
    sim = make(cfg, occ)
    wall = 100 * s
    # 0 plain progress; 1 goal reached; 2 collision; 3 goal and collision;
    # 4 horizon reached with no event
    put(sim, 0, x=2.0, y=2.0, th=0.0, gx=4.0, gy=2.0, dprev=f32(2.1), t=5)
    put(sim, 1, x=2.0, y=2.0, th=0.0, gx=2.1, gy=2.0, dprev=f32(0.5), t=5)
    put(sim, 2, x=wall - 0.2, y=3.0, th=0.0, gx=2.0, gy=3.0, dprev=f32(3.0), t=5)
    put(sim, 3, x=wall - 0.2, y=4.0, th=0.0, gx=wall - 0.15, gy=4.0, dprev=f32(0.3), t=5)
    put(sim, 4, x=1.0, y=8.0, th=0.0, gx=1.0, gy=1.0, dprev=f32(7.0), t=199)
    act = np.array([[-1, 0], [-1, 0], [1, 0], [1, 0], [-1, 0]], np.float32)
    st0 = sim.get_state()
    o = sim.step(act)
    assert list(o["terminated"]) == [0, 1, 1, 1, 0]
    assert list(o["truncated"]) == [0, 0, 0, 0, 1]
    assert list(o["collision"]) == [0, 0, 1, 1, 0]
    assert list(o["goal"]) == [0, 1, 0, 1, 0]
    assert o["reward"][1] == 10.0 and o["reward"][2] == -10.0 and o["reward"][3] == 10.0
    d0 = f32(math.hypot(4.0 - 2.0, 0.0))
    assert o["reward"][0] == f32(2.0 * (float(st0["dprev"][0]) - d0))
    d4 = f32(7.0)
    assert o["reward"][4] == f32(2.0 * (7.0 - d4))
    assert list(o["reset"]) == [0, 1, 1, 1, 1]
    assert not np.any(o["terminated"] & o["truncated"])


def test_idle_robot_truncates_exactly_at_horizon():
    sim = make(base_cfg(num_envs=1, horizon=200))
    put(sim, 0, x=5.0, y=5.0, th=0.0, gx=8.0, gy=5.0, dprev=3.0, t=0)
    act = np.array([[-1.0, 0.0]], np.float32)
    for n in range(1, 201):
        o = sim.step(act)
        assert o["terminated"][0] == 0
        assert o["truncated"][0] == (1 if n == 200 else 0)
    assert sim.get_state()["t"][0] == 0


def test_pooling_is_sector_min():
    w = configs.build_workload("c2", num_envs=64)
    sim = oracle.OracleSim(w["cfg"], w["maps"], w["res"], w["env_map"])
    sim.reset()
    o = sim.step(configs.uniform_actions(1, 64)[0])
    K, m = sim.K, sim.m
    per = K // m
    live = o["reset"] == 0
    rg = o["ranges"][live].reshape(-1, m, per)
    pooled = o["obs"][live, :m]
    assert np.all(pooled[:, :, None] <= rg)
    assert np.all(np.any(pooled[:, :, None] == rg, axis=2))
    assert np.all((o["ranges"] >= 0) & (o["ranges"] <= np.float32(6.0)))


def _check_reset_rows(sim, obs, fallback, rows):
    st = sim.get_state()
    occ = sim.maps.maps
    for e in rows:
        k = int(sim.env_map[e])
        s = float(sim.maps.res[k])
        x, y, th = float(st["x"][e]), float(st["y"][e]), float(st["th"][e])
        gx, gy = float(st["gx"][e]), float(st["gy"][e])
        if sim.cfg_dict["footprint"] == 0:
            assert not brute_disc(occ[k], s, x, y, f32(sim.cfg_dict["radius_m"]))
            rc = f32(sim.cfg_dict["radius_m"])
        else:
            hit, amb = brute_rect(occ[k], s, x, y, th, f32(sim.cfg_dict["length_m"]),
                                  f32(sim.cfg_dict["width_m"]))
            assert not hit
            rc = math.hypot(f32(sim.cfg_dict["length_m"]) / 2, f32(sim.cfg_dict["width_m"]) / 2)
        assert not brute_disc(occ[k], s, gx, gy, rc)
        if not (fallback[e] & 2):
            assert math.hypot(gx - x, gy - y) >= f32(sim.cfg_dict["goal_min_dist_m"])
        assert st["t"][e] == 0 and st["v"][e] == 0 and st["w"][e] == 0
        m = sim.m
        assert obs[e, m + 2] == 0 and obs[e, m + 3] == 0
        assert st["dprev"][e] == obs[e, m]


@pytest.mark.parametrize("wl", ["c1", "c3"])
def test_reset_invariants(wl):
    w = configs.build_workload(wl, num_envs=24)
    sim = oracle.OracleSim(w["cfg"], w["maps"], w["res"], w["env_map"])
    obs, fb = sim.reset()
    _check_reset_rows(sim, obs, fb, range(24))
    acts = configs.uniform_actions(60, 24, seed=3)
    seen = 0
    for t in range(60):
        o = sim.step(acts[t])
        rows = np.nonzero(o["reset"])[0]
        _check_reset_rows(sim, o["obs"], o["fallback"], rows)
        seen += len(rows)
        # the final observation is the pre-reset one: pooled debug ranges
        m, per = sim.m, sim.K // sim.m
        for e in rows:
            pooled = o["ranges"][e].reshape(m, per).min(axis=1)
            assert np.array_equal(o["final_obs"][e, :m], pooled)
    assert seen > 0


def test_reset_mask_and_determinism():
    w = configs.build_workload("c2", num_envs=32)
    a = oracle.OracleSim(w["cfg"], w["maps"], w["res"], w["env_map"])
    b = oracle.OracleSim(w["cfg"], w["maps"], w["res"], w["env_map"])
    a.reset()
    b.reset()
    for k in oracle.STATE_KEYS:
        assert np.array_equal(a.state[k], b.state[k])
    before = a.get_state()
    mask = np.zeros(32, np.uint8)
    mask[[3, 17]] = 1
    a.reset(mask)
    after = a.get_state()
    for k in oracle.STATE_KEYS:
        same = np.ones(32, bool)
        same[[3, 17]] = False
        assert np.array_equal(before[k][same], after[k][same])
    assert after["ep"][3] == before["ep"][3] + 1
    assert (after["x"][3], after["y"][3]) != (before["x"][3], before["y"][3])
    c = oracle.OracleSim(dict(w["cfg"], seed=12345), w["maps"], w["res"], w["env_map"])
    c.reset()
    assert not np.array_equal(c.state["x"], b.state["x"])


def test_fallback_when_free_space_is_tiny():
    # 40x40 cells of 0.1 m, solid except a 5x5-cell pocket: random attempts
    # rarely fit the 0.18 m disc and no goal can be 1 m away, so the free-cell
    # fallback is taken; its poses must still be valid.
    occ = np.ones((40, 40), np.uint8)
    occ[10:15, 20:25] = 0
    cfg = base_cfg(num_envs=16, max_range_m=2.0)
    sim = make(cfg, occ, res=0.1)
    obs, fb = sim.reset()
    assert np.all(fb & 2)
    assert np.any(fb & 1)
    _check_reset_rows(sim, obs, fb, range(16))


def test_deferred_reset_then_masked_reset_equals_the_plain_step():
    # an env whose reset is deferred keeps its post-step state and counters;
    # resetting exactly the deferred envs afterwards draws the same poses
    # (the draw depends only on env, episode and attempt), so the two-part
    # step equals the plain one, and envs without a bin are reset as usual
    w = configs.build_workload("c2", num_envs=48)
    a = oracle.OracleSim(w["cfg"], w["maps"], w["res"], w["env_map"])
    b = oracle.OracleSim(w["cfg"], w["maps"], w["res"], w["env_map"])
    a.reset()
    st = a.get_state()
    st["t"][::3] = 199  # a third of the envs truncate in the next step
    a.set_state(st)
    b.set_state(st)
    bins = np.where(np.arange(48) % 2 == 0, np.arange(48) % 8, -1).astype(np.int32)
    act = configs.uniform_actions(1, 48, seed=9)[0]
    oa = a.step(act)
    ob = b.step(act, defer_bin=bins)
    for k in ("terminated", "truncated", "reward", "collision", "reset", "final_obs"):
        assert np.array_equal(oa[k], ob[k]), k
    done = ob["reset"].astype(bool)
    deferred = done & (bins >= 0)
    assert deferred.sum() >= 4 and (done & (bins < 0)).sum() >= 4
    after = b.get_state()
    # deferred envs: the post-step pose, episode counter unchanged
    assert np.array_equal(after["ep"][deferred], st["ep"][deferred])
    assert np.all(after["t"][deferred] == st["t"][deferred] + 1)
    # every other env: the plain step's state and observation
    keep = ~deferred
    for k in oracle.STATE_KEYS:
        assert np.array_equal(after[k][keep], a.state[k][keep]), k
    assert np.array_equal(ob["obs"][keep], oa["obs"][keep])
    obs2, _ = b.reset(deferred.astype(np.uint8))
    for k in oracle.STATE_KEYS:
        assert np.array_equal(b.state[k], a.state[k]), k
    assert np.array_equal(obs2[deferred], oa["obs"][deferred])
