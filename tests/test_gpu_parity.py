"""GPU parity: the HIP step (fused and plain mappings, through the C ABI)
against the CPU oracle, teacher-forced from identical states each step."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2606_15846_amd import navsim
from paper_2606_15846_amd.navsim import NAVSIM_KERNEL_FUSED, NAVSIM_KERNEL_PLAIN, NavSim
from tests.parity import compare_step, gpu_step
from workloads import configs

pytestmark = pytest.mark.gpu
KERNELS = {"fused": NAVSIM_KERNEL_FUSED, "plain": NAVSIM_KERNEL_PLAIN}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_pair(cfg, maps, res, env_map, profiles=None):
    sim = NavSim(cfg, maps, res, env_map, device=0, profiles=profiles)
    ref = oracle.OracleSim(cfg, maps, res, env_map, profiles=profiles)
    return sim, ref


def run_teacher_forced(sim, ref, steps, kernel, seed=42, threads=16, label=""):
    obs = sim.reset()
    ref_obs, _ = ref.reset(threads=threads)
    torch.cuda.synchronize()
    st = sim.get_state()
    for k in oracle.STATE_KEYS:
        assert np.array_equal(st[k], ref.state[k]), f"{label}: reset state {k} differs"
    acts = configs.uniform_actions(steps, ref.N, seed=seed)
    totals = dict(rays=0, grazing=0, grazing_mismatch=0, resets=0, visits=0)
    for t in range(steps):
        # the oracle runs free on its own state; compare_step asserts that
        # the two states stay bitwise equal after every step
        g, gst = gpu_step(sim, acts[t], kernel)
        r = ref.step(acts[t], threads=threads)
        c = compare_step(g, r, gst, ref, label=f"{label} step {t}")
        for k in totals:
            totals[k] += c[k]
    say(f"{label}: {totals}")
    return totals


@pytest.mark.parametrize("kname", ["fused", "plain"])
def test_c1_full_rollout(kname):
    say(f"c1 rollout 16 envs x 200 steps, kernel={kname}")
    w = configs.build_workload("c1")
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"])
    tot = run_teacher_forced(sim, ref, 200, KERNELS[kname], label=f"c1/{kname}")
    assert tot["resets"] > 0
    sim.close()


def test_c2_full_size_fused():
    say("c2 4096 envs x 360 beams, 16 maps 128^2, fused, 4 steps")
    w = configs.build_workload("c2")
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"])
    tot = run_teacher_forced(sim, ref, 4, NAVSIM_KERNEL_FUSED, label="c2/fused")
    assert tot["grazing"] < 0.01 * tot["rays"]
    sim.close()


def test_c2_plain_subset():
    say("c2 maps, 256 envs, plain, 3 steps")
    w = configs.build_workload("c2", num_envs=256)
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"])
    run_teacher_forced(sim, ref, 3, NAVSIM_KERNEL_PLAIN, label="c2/plain")
    sim.close()


@pytest.mark.parametrize("walk", [0, 1, 2, 3, 4, 5])
def test_walk_variants_against_oracle(walk):
    say(f"walk = {walk} (0 chunked groups, 1 runs, 2 byte-per-cell map, 3 claim walk, 4 claim "
        f"walk on bytes, 5 claim walk over runs on the bitmap and its transpose): c2 full size "
        f"and c3 maps, fused, teacher-forced")
    w = configs.build_workload("c2")
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"])
    sim.set_tuning(4, 48, 4, 0, walk)
    run_teacher_forced(sim, ref, 3, NAVSIM_KERNEL_FUSED, label=f"c2/walk{walk}")
    sim.close()
    w = configs.build_workload("c3", num_envs=1024)
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"])
    big = walk in (2, 4)  # the byte copy of a 256^2 map needs 1024-thread workgroups' LDS
    sim.set_tuning(4 if big else 2, 40, 8, 0, walk, threads=1024 if big else 256)
    run_teacher_forced(sim, ref, 3, NAVSIM_KERNEL_FUSED, label=f"c3/walk{walk}")
    sim.close()


def test_run_walk_on_grid_lines_corners_and_axis_rays():
    """Origins exactly on grid lines and corners (1/16 m cells: the coordinates
    are exact in float), heading 0 with 360 beams over the full circle (the
    axis-parallel and 45-degree rays among them), 8 m range (runs far longer
    than one 31-cell window): the run walk on the bitmap and its transpose
    (walk 5) gives bitwise the hits, visits and ranges of the claim walks on
    the bitmap (3) and on bytes (4), of the chunked run walk (1) and of the
    plain kernel's cell-by-cell walk; non-grazing rays against the oracle."""
    say("run walk: 512 envs on grid corners and lines of a 1/16 m map, axis and 45-degree "
        "rays, walks 5 / 3 / 4 / 1 / plain")
    from workloads import maps as gm
    res = 0.0625
    occ = gm.gen_rect_disc_map(23, w=200, h=180, res=res)
    N = 512
    cfg = configs.make_config(num_envs=N, num_beams=360, num_sectors=36, fov_rad=2 * math.pi,
                              max_range_m=8.0, dt_s=0.1, footprint=0, radius_m=0.1,
                              v_min=0.0, v_max=0.5, w_min=-1.0, w_max=1.0)
    env_map = np.zeros(N, np.int32)
    rng = np.random.default_rng(7)
    free = np.argwhere(occ == 0)
    pick = free[rng.choice(len(free), N, replace=False)]
    offs = np.array([(0, 0), (0.5, 0), (0, 0.5), (0.5, 0.5), (0.25, 0), (0, 0.75)])
    o = offs[np.arange(N) % len(offs)]
    x = ((pick[:, 1] + o[:, 0]) * res).astype(np.float32)
    y = ((pick[:, 0] + o[:, 1]) * res).astype(np.float32)
    assert np.array_equal(x.astype(np.float64) / res % 0.25, np.zeros(N))  # on the grid
    th = np.where(np.arange(N) % 4 == 3, np.float32(0.4), np.float32(0.0)).astype(np.float32)
    acts = np.tile(np.array([-1.0, 0.0], np.float32), (N, 1))  # v = 0, w = 0: pose kept
    runs = []
    for kernel, walk, te, thr in [(NAVSIM_KERNEL_FUSED, 5, 8, 256),
                                  (NAVSIM_KERNEL_FUSED, 5, 32, 1024),
                                  (NAVSIM_KERNEL_FUSED, 3, 8, 256),
                                  (NAVSIM_KERNEL_FUSED, 4, 16, 1024),
                                  (NAVSIM_KERNEL_FUSED, 1, 4, 256),
                                  (NAVSIM_KERNEL_PLAIN, 0, 4, 256)]:
        sim, ref = make_pair(cfg, [occ], [res], env_map)
        sim.set_tuning(te, 40, 8, 0, walk, threads=thr)
        sim.reset()
        torch.cuda.synchronize()
        st = sim.get_state()
        st["x"][:] = x
        st["y"][:] = y
        st["th"][:] = th
        st["t"][:] = 0
        sim.set_state(st)
        g, gst = gpu_step(sim, acts, kernel)
        kept = ~g["reset"].astype(bool)
        assert np.array_equal(gst["x"][kept], x[kept]) and np.array_equal(gst["th"][kept], th[kept])
        if walk == 5 and te == 8:
            ref.set_state(st)
            r = ref.step(acts, threads=16)
            rep = compare_step(g, r, gst, ref, label="run walk on the grid")
            say(f"grazing rays {rep['grazing']} of {N * 360}; longest walk "
                f"{int(g['visits'].max())} cells")
            assert int(g["visits"].max()) > 64
        runs.append(g)
        sim.close()
    ended = runs[0]["reset"].astype(bool)
    for i, other in enumerate(runs[1:]):
        for k in ("ranges", "hits", "visits", "obs", "reward", "terminated", "reset"):
            assert np.array_equal(runs[0][k], other[k]), (i + 1, k)
        assert np.array_equal(runs[0]["final_obs"][ended], other["final_obs"][ended]), i + 1


def test_c3_full_size_fused():
    say("c3 full size: 16384 envs, 64 rooms maps 256^2, rectangle, 720 beams, 2 steps")
    w = configs.build_workload("c3")
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"])
    tot = run_teacher_forced(sim, ref, 2, NAVSIM_KERNEL_FUSED, label="c3-full/fused")
    assert tot["grazing"] < 0.01 * tot["rays"]
    sim.close()


def test_c5_full_size_fused():
    say("c5 full size: 65536 envs, 64 rooms maps 256^2, 360 beams, 2 steps")
    w = configs.build_workload("c5")
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"])
    tot = run_teacher_forced(sim, ref, 2, NAVSIM_KERNEL_FUSED, label="c5-full/fused")
    assert tot["grazing"] < 0.01 * tot["rays"]
    sim.close()


def test_c3_rect_reverse_fused():
    say("c3 maps 256^2, rectangle footprint, 720 beams, 2048 envs, fused, 3 steps")
    w = configs.build_workload("c3", num_envs=2048)
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"])
    run_teacher_forced(sim, ref, 3, NAVSIM_KERNEL_FUSED, label="c3/fused")
    sim.close()


def test_c4_mixed_profiles_full_size_fused():
    say("c4 32768 envs, 128 uneven maps, per-map K and footprint, fused, 2 steps")
    w = configs.build_workload("c4")
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"], w["profiles"])
    tot = run_teacher_forced(sim, ref, 2, NAVSIM_KERNEL_FUSED, label="c4/fused")
    assert tot["grazing"] < 0.01 * tot["rays"]
    sim.close()


def test_c4_full_size_launch_shapes_agree():
    # launch shapes the C4 line of the bench may time, against the per-tile
    # 256-thread launch that the test above holds to the oracle; 1024 threads
    # take more than 64 KiB of LDS per workgroup
    say("c4 full size: persistent workgroups and 512 / 1024 threads == per-tile, 3 steps")
    w = configs.build_workload("c4")
    acts = torch.from_numpy(configs.uniform_actions(3, w["cfg"]["num_envs"], seed=5)).cuda()
    runs = []
    for te, pe, th, wk, bal in [(8, 0, 256, 0, 0), (8, 4, 256, 0, 0), (4, 1, 256, 0, 0),
                                (16, 16, 256, 0, 0), (8, 0, 512, 0, 0), (16, 0, 1024, 0, 0),
                                (4, 0, 1024, 0, 0), (4, 0, 512, 3, 0), (8, 2, 256, 3, 0),
                                (16, 0, 512, 3, 1), (32, 0, 1024, 3, 1), (8, 3, 256, 3, 1),
                                (16, 0, 512, 5, 1), (32, 0, 512, 5, 1), (8, 0, 256, 5, 1),
                                (8, 3, 256, 5, 0), (32, 0, 1024, 5, 1)]:
        sim = NavSim(w["cfg"], w["maps"], w["res"], w["env_map"], device=0,
                     profiles=w["profiles"])
        sim.set_tuning(te, 48, 8, walk=wk, persist=pe, threads=th, balance=bal)
        outs = [sim.reset().cpu().numpy().copy()]
        for t in range(3):
            o, r, te_, tr, info = sim.step(acts[t])
            fo = info["final_obs"]
            done = (te_ | tr).cpu().numpy().astype(bool)
            outs += [o.cpu().numpy().copy(), r.cpu().numpy().copy(), done,
                     fo.cpu().numpy()[done].copy()]
        st = sim.get_state()
        outs += [st[k] for k in oracle.STATE_KEYS]
        runs.append(outs)
        sim.close()
    for other in runs[1:]:
        for i, (a, b) in enumerate(zip(runs[0], other)):
            assert np.array_equal(a, b), i


def _mixed_small(num_envs=96):
    """Six maps of different sizes, one of each beam count and both footprints."""
    from workloads import maps as gm
    occ = [gm.gen_rect_disc_map(11, w=70, h=50, res=0.05),
           gm.gen_rooms_map(12, w=120, h=97, res=0.05),
           gm.gen_rect_disc_map(13, w=33, h=140, res=0.05),
           gm.gen_rooms_map(14, w=200, h=180, res=0.05),
           gm.gen_rect_disc_map(15, w=96, h=96, res=0.05),
           gm.gen_rect_map(16, w=64, h=64)]
    res = [0.05] * 5 + [0.1]
    prof = [dict(num_beams=180, footprint=0, radius_m=0.18),
            dict(num_beams=1080, footprint=1, length_m=0.70, width_m=0.31),
            dict(num_beams=360, footprint=1, length_m=0.80, width_m=0.41),
            dict(num_beams=720, footprint=0, radius_m=0.2),
            dict(num_beams=30, footprint=0, radius_m=0.12),
            dict(num_beams=90, footprint=1, length_m=0.5, width_m=0.3)]
    cfg = configs.make_config(num_envs=num_envs, num_beams=1080, num_sectors=30,
                              fov_rad=2 * math.pi, max_range_m=8.0, dt_s=0.1, footprint=0,
                              radius_m=0.18, v_min=-0.5, v_max=0.5, w_min=-1.0, w_max=1.0)
    # interleaved, so tiles are formed from envs that are not contiguous
    env_map = (np.arange(num_envs) * 7 % len(occ)).astype(np.int32)
    return cfg, occ, res, env_map, prof


@pytest.mark.parametrize("kname", ["fused", "plain"])
def test_mixed_profiles_rollout(kname):
    say(f"mixed profiles: 6 maps, K 30..1080, disc+rect, 96 envs, 40 steps, kernel={kname}")
    cfg, occ, res, env_map, prof = _mixed_small()
    sim, ref = make_pair(cfg, occ, res, env_map, prof)
    tot = run_teacher_forced(sim, ref, 40, KERNELS[kname], seed=9, label=f"mixed/{kname}")
    assert tot["resets"] > 0
    sim.close()


def test_mixed_profiles_launch_shapes_agree():
    say("mixed profiles: fused under every tile size == plain, bitwise, 5 steps")
    cfg, occ, res, env_map, prof = _mixed_small(num_envs=150)
    acts = configs.uniform_actions(5, cfg["num_envs"], seed=33)
    runs = []
    F = NAVSIM_KERNEL_FUSED
    for kernel, te, pe, thr, walk in [
            (NAVSIM_KERNEL_PLAIN, 4, 0, 256, 0), (F, 4, 0, 256, 0), (F, 8, 0, 256, 0),
            (F, 16, 0, 256, 0), (F, 4, 3, 256, 0), (F, 2, 16, 256, 0), (F, 8, 0, 512, 0),
            (F, 16, 0, 1024, 0), (F, 4, 0, 256, 2), (F, 8, 2, 1024, 2), (F, 4, 0, 256, 3),
            (F, 16, 0, 1024, 4), (F, 4, 0, 256, 5), (F, 16, 2, 1024, 5), (F, 1, 0, 256, 5)]:
        sim = NavSim(cfg, occ, res, env_map, device=0, profiles=prof)
        sim.set_tuning(te, 48, 4, walk=walk, persist=pe, threads=thr)
        sim.reset()
        runs.append([gpu_step(sim, acts[t], kernel) for t in range(5)])
        sim.close()
    for other in runs[1:]:
        for (ga, sa), (gb, sb) in zip(runs[0], other):
            for k in ga:
                assert np.array_equal(ga[k], gb[k]) or k == "final_obs", k
            for k in oracle.STATE_KEYS:
                assert np.array_equal(sa[k], sb[k]), k


@pytest.mark.parametrize("te", [1, 2, 4])
def test_small_tiles_with_an_odd_sector_count(te):
    # m = 9: a tile's sector pool is 2 E m words, padded to keep the LDS
    # regions after it aligned
    say(f"odd m = 9, K = 99, tile_envs = {te}: fused == plain == oracle")
    from workloads import maps as gm
    occ = gm.gen_rect_disc_map(17, w=80, h=72, res=0.05)
    cfg = _small_cfg(num_envs=21, num_beams=99, num_sectors=9)
    env_map = np.zeros(21, np.int32)
    sim, ref = make_pair(cfg, [occ], [0.05], env_map)
    sim.set_tuning(te, 48, 4)
    run_teacher_forced(sim, ref, 12, NAVSIM_KERNEL_FUSED, seed=3, label=f"m9/E{te}")
    sim.close()


def test_profile_validation_on_device():
    cfg, occ, res, env_map, prof = _mixed_small(num_envs=12)
    for bad in [dict(num_beams=1110), dict(num_beams=100), dict(num_beams=0),
                dict(footprint=3), dict(footprint=0, radius_m=0.0),
                dict(footprint=1, length_m=0.5, width_m=-1.0)]:
        p2 = [dict(q) for q in prof]
        p2[2].update(bad)
        with pytest.raises(navsim.NavsimError) as ei:
            NavSim(cfg, occ, res, env_map, device=0, profiles=p2)
        assert ei.value.status == -1 and "map 2" in str(ei.value), bad
    with pytest.raises(ValueError):
        NavSim(cfg, occ, res, env_map, device=0, profiles=prof[:3])


@pytest.mark.parametrize("kname", ["fused", "plain"])
def test_march_scan_mode_against_oracle(kname):
    say(f"fixed-step march (0.03 m), c2 maps, 512 envs, 4 steps, kernel={kname}")
    w = configs.build_workload("c2", num_envs=512)
    cfg = dict(w["cfg"], scan_mode=1, march_step_m=0.03)
    sim, ref = make_pair(cfg, w["maps"], w["res"], w["env_map"])
    sim.set_scan(navsim.NAVSIM_SCAN_MARCH, 0.03)
    tot = run_teacher_forced(sim, ref, 4, KERNELS[kname], label=f"march/{kname}")
    assert tot["grazing"] < 1e-3 * tot["rays"]
    sim.close()


def test_march_mixed_profiles_and_launch_shapes():
    say("fixed-step march on mixed profiles: fused (tile 4, 16) == plain, and vs oracle")
    cfg, occ, res, env_map, prof = _mixed_small(num_envs=60)
    cfg = dict(cfg, scan_mode=1, march_step_m=0.05)
    sim, ref = make_pair(cfg, occ, res, env_map, prof)
    sim.set_scan(navsim.NAVSIM_SCAN_MARCH, 0.05)
    run_teacher_forced(sim, ref, 6, NAVSIM_KERNEL_FUSED, seed=4, label="march-mixed")
    acts = configs.uniform_actions(3, 60, seed=8)
    runs = []
    # walks 4 and 5 (claim walks) apply to the exact traversal only: the march
    # keeps its chunked path under them
    for kernel, te, wk in [(NAVSIM_KERNEL_PLAIN, 4, 0), (NAVSIM_KERNEL_FUSED, 4, 0),
                           (NAVSIM_KERNEL_FUSED, 16, 0), (NAVSIM_KERNEL_FUSED, 4, 4),
                           (NAVSIM_KERNEL_FUSED, 4, 5)]:
        s2 = NavSim(cfg, occ, res, env_map, device=0, profiles=prof)
        s2.set_scan(navsim.NAVSIM_SCAN_MARCH, 0.05)
        s2.set_tuning(te, 40, 2, walk=wk)
        s2.reset()
        runs.append([gpu_step(s2, acts[t], kernel) for t in range(3)])
        s2.close()
    for other in runs[1:]:
        for (ga, sa), (gb, sb) in zip(runs[0], other):
            for k in ga:
                assert np.array_equal(ga[k], gb[k]) or k == "final_obs", k
    with pytest.raises(navsim.NavsimError):
        sim.set_scan(7, 0.03)
    with pytest.raises(navsim.NavsimError):
        sim.set_scan(navsim.NAVSIM_SCAN_MARCH, 0.0)
    sim.close()


def _small_cfg(**kw):
    c = configs.make_config(num_envs=13, num_beams=100, num_sectors=10, fov_rad=2 * math.pi,
                            max_range_m=2.5, dt_s=0.1, footprint=0, radius_m=0.18,
                            v_min=-0.5, v_max=0.5, w_min=-1.0, w_max=1.0)
    c.update(kw)
    return c


@pytest.mark.parametrize("case", ["ragged", "many_sectors", "fov270", "rect_noborder",
                                  "single_env", "long_range", "max_beams"])
@pytest.mark.parametrize("kname", ["fused", "plain"])
def test_edge_configs(case, kname):
    say(f"edge config {case}, kernel={kname}")
    from workloads import maps as gm
    occ = gm.gen_rect_disc_map(7, w=90, h=70, res=0.05)
    cfg = _small_cfg()
    if case == "many_sectors":
        cfg.update(num_beams=130, num_sectors=130)
    elif case == "fov270":
        cfg.update(fov_rad=math.radians(270.0), num_beams=1080, num_sectors=30, max_range_m=20.0)
    elif case == "rect_noborder":
        occ = (np.random.default_rng(3).random((60, 75)) < 0.003).astype(np.uint8)
        cfg.update(footprint=1, length_m=0.8, width_m=0.41)
    elif case == "single_env":
        cfg.update(num_envs=1)
    elif case == "long_range":
        cfg.update(max_range_m=50.0, num_beams=64, num_sectors=8)
    elif case == "max_beams":
        # the largest beam count: the claim index and the beam's sector come
        # from multiply-shift quotients whose exact range ends here
        cfg.update(num_beams=4096, num_sectors=64)
    maps = [occ, occ[::-1].copy()]
    env_map = (np.arange(cfg["num_envs"]) % 2).astype(np.int32)
    sim, ref = make_pair(cfg, maps, [0.05, 0.05], env_map)
    run_teacher_forced(sim, ref, 25, KERNELS[kname], seed=5, label=f"{case}/{kname}")
    sim.close()


def _crowded_map():
    # mostly occupied: three rooms hold ~22 % of the cells, and a disc of
    # r 0.18 m fits around ~11 % of them
    occ = np.ones((80, 100), np.uint8)
    occ[8:30, 8:40] = 0
    occ[48:72, 55:92] = 0
    occ[30:42, 68:82] = 0
    return occ


@pytest.mark.parametrize("case", ["tries5", "tries12", "tries40", "rect20"])
@pytest.mark.parametrize("kname", ["fused", "plain"])
def test_crowded_map_reset_attempts(case, kname):
    """Start and goal draws on a crowded map need many attempts: the first
    success often comes after attempt 8 or 16 (the fused step's later passes)
    or never (the free-cell fallback), with fewer attempts than one pass (5),
    between one and two passes (12), many (40), and with a rectangle."""
    say(f"crowded map, {case}, kernel={kname}")
    occ = _crowded_map()
    tries = {"tries5": 5, "tries12": 12, "tries40": 40, "rect20": 20}[case]
    cfg = _small_cfg(num_envs=40, reset_max_tries=tries, goal_min_dist_m=1.0)
    if case == "rect20":
        cfg.update(footprint=1, length_m=0.5, width_m=0.3)
    maps = [occ, occ[::-1].copy()]
    env_map = (np.arange(cfg["num_envs"]) % 2).astype(np.int32)
    _, fb = oracle.OracleSim(cfg, maps, [0.05, 0.05], env_map).reset(threads=16)
    say(f"oracle reset: start fallbacks {int(((fb & 1) != 0).sum())}, "
        f"goal fallbacks {int(((fb & 2) != 0).sum())} of {cfg['num_envs']}")
    if tries <= 12:
        assert (fb != 0).any()
    sim, ref = make_pair(cfg, maps, [0.05, 0.05], env_map)
    tot = run_teacher_forced(sim, ref, 20, KERNELS[kname], seed=9, label=f"crowded {case}/{kname}")
    assert tot["resets"] > 0
    sim.close()


def test_pose_outside_map_and_inside_obstacle():
    say("poses outside the map / inside an obstacle")
    occ = np.zeros((40, 40), np.uint8)
    occ[20:25, 20:25] = 1
    cfg = _small_cfg(num_envs=4, num_beams=64, num_sectors=8)
    sim, ref = make_pair(cfg, [occ], [0.05], np.zeros(4, np.int32))
    sim.reset()
    ref.reset()
    torch.cuda.synchronize()
    st = ref.get_state()
    st["x"][:] = [-0.3, 1.1, 2.5, 1.0]
    st["y"][:] = [0.5, 1.1, 0.5, 1.0]
    st["v"][:] = 0.0
    sim.set_state(st)
    ref.set_state(st)
    act = np.zeros((4, 2), np.float32)
    act[:, 0] = 0.0   # v = 0 (bounds -0.5..0.5)
    g, gst = gpu_step(sim, act, NAVSIM_KERNEL_FUSED)
    r = ref.step(act)
    compare_step(g, r, gst, ref, label="outside/inside")
    assert r["collision"][0] and r["collision"][1] and r["collision"][2]
    assert np.all(g["hits"][0] == -2) and np.all(g["ranges"][0] == 0)
    assert np.all(g["ranges"][1] == 0)
    sim.close()


def test_fused_equals_plain_bitwise():
    say("fused vs plain bitwise, c2 maps, 512 envs, 5 steps")
    w = configs.build_workload("c2", num_envs=512)
    a = NavSim(w["cfg"], w["maps"], w["res"], w["env_map"], device=0)
    b = NavSim(w["cfg"], w["maps"], w["res"], w["env_map"], device=0)
    a.reset()
    b.reset()
    acts = configs.uniform_actions(5, 512, seed=9)
    for t in range(5):
        ga, sa = gpu_step(a, acts[t], NAVSIM_KERNEL_FUSED)
        gb, sb = gpu_step(b, acts[t], NAVSIM_KERNEL_PLAIN)
        for k in ga:
            assert np.array_equal(ga[k], gb[k]) or k == "final_obs", k
        for k in oracle.STATE_KEYS:
            assert np.array_equal(sa[k], sb[k]), k
    a.close()
    b.close()


@pytest.mark.parametrize("walk", [3, 4, 5])
def test_every_env_resets_every_step(walk):
    """Horizon 1: every env ends and is reset in every step, so a tile's
    reset jobs (drawn while the claim walk already runs on the main jobs, the
    final observations here) are as many as its envs and rays of unpublished
    reset jobs are claimed; teacher-forced against the oracle."""
    say(f"horizon 1, walk {walk}: every env resets every step, 32-env tiles, c2 maps, 512 envs")
    w = configs.build_workload("c2", num_envs=512)
    cfg = dict(w["cfg"], horizon=1)
    sim, ref = make_pair(cfg, w["maps"], w["res"], w["env_map"])
    sim.set_tuning(32, 40, 16, 0, walk, threads=1024 if walk == 4 else 512)
    tot = run_teacher_forced(sim, ref, 3, NAVSIM_KERNEL_FUSED, label=f"horizon1/walk{walk}")
    assert tot["resets"] == 3 * 512
    sim.close()


def test_determinism_and_checkpoint():
    say("determinism + checkpoint/resume, c2 maps, 256 envs")
    w = configs.build_workload("c2", num_envs=256)
    acts = torch.from_numpy(configs.uniform_actions(100, 256, seed=11)).cuda()

    def run(sim, t0, t1):
        for t in range(t0, t1):
            sim.step(acts[t])
        torch.cuda.synchronize()
        return sim.obs.cpu().numpy().copy(), sim.get_state()

    a = NavSim(w["cfg"], w["maps"], w["res"], w["env_map"], device=0)
    a.reset()
    oa, sa = run(a, 0, 100)
    b = NavSim(w["cfg"], w["maps"], w["res"], w["env_map"], device=0)
    b.reset()
    _, mid = run(b, 0, 50)
    b.close()
    c = NavSim(w["cfg"], w["maps"], w["res"], w["env_map"], device=0)
    c.set_state(mid)
    oc, sc = run(c, 50, 100)
    assert np.array_equal(oa, oc)
    for k in oracle.STATE_KEYS:
        assert np.array_equal(sa[k], sc[k]), k
    a.close()
    c.close()


def test_reset_mask_leaves_other_rows():
    say("masked reset")
    w = configs.build_workload("c2", num_envs=64)
    sim, ref = make_pair(w["cfg"], w["maps"], w["res"], w["env_map"])
    sim.reset()
    ref.reset()
    torch.cuda.synchronize()
    before = sim.obs.cpu().numpy().copy()
    mask = np.zeros(64, np.uint8)
    mask[[0, 5, 63]] = 1
    sim.reset(torch.from_numpy(mask).cuda())
    ro, _ = ref.reset(mask)
    torch.cuda.synchronize()
    after = sim.obs.cpu().numpy()
    keep = mask == 0
    assert np.array_equal(before[keep], after[keep])
    st = sim.get_state()
    for k in oracle.STATE_KEYS:
        assert np.array_equal(st[k], ref.state[k]), k
    assert np.abs(after[mask == 1] - ro[mask == 1]).max() <= 1e-4
    sim.close()


def test_api_errors_on_device():
    say("API error paths on the device")
    w = configs.build_workload("c1")
    cfg = w["cfg"]
    h = navsim.navsim_create(cfg, 0)
    obs = torch.zeros(16, cfg["num_sectors"] + 4, device="cuda")
    act = torch.zeros(16, 2, device="cuda")
    r = torch.zeros(16, device="cuda")
    u8 = torch.zeros(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(navsim.NavsimError) as ei:
        navsim.navsim_step(h, act, obs, r, u8, u8)
    assert ei.value.status == -3
    with pytest.raises(navsim.NavsimError) as ei:
        navsim.navsim_load_maps(h, w["maps"], w["res"], np.full(16, 3, np.int32))
    assert ei.value.status == -1
    full = np.ones((20, 20), np.uint8)
    with pytest.raises(navsim.NavsimError) as ei:
        navsim.navsim_load_maps(h, [full], [0.1], np.zeros(16, np.int32))
    assert ei.value.status == -4
    navsim.navsim_load_maps(h, w["maps"], w["res"], w["env_map"])
    with pytest.raises(navsim.NavsimError) as ei:
        navsim.navsim_reset(h, u8, obs)
    assert ei.value.status == -3
    navsim.navsim_reset(h, None, obs)
    navsim.navsim_step(h, act, obs, r, u8, u8)
    torch.cuda.synchronize()
    # launch-shape validation: each bad field alone; the handle keeps its shape
    before = navsim.navsim_get_tuning(h)
    base = dict(tile_envs=4, refill_at=48, groups=4, ray_slots=0, walk=0, persist=0, threads=256)
    for bad in [dict(tile_envs=3), dict(refill_at=64), dict(groups=0), dict(ray_slots=100),
                dict(walk=6), dict(persist=65), dict(threads=384), dict(tile_envs=32),
                dict(balance=2)]:
        with pytest.raises(navsim.NavsimError) as ei:
            navsim.navsim_set_tuning(h, **dict(base, **bad))
        assert ei.value.status == -1, bad
    assert navsim.navsim_get_tuning(h) == before
    navsim.navsim_destroy(h)


def test_launch_shape_does_not_change_results():
    say("tuning invariance: tile_envs x refill_at x groups, c2 maps, 600 envs, 3 steps")
    w = configs.build_workload("c2", num_envs=600)
    acts = configs.uniform_actions(3, 600, seed=21)
    ref_out = None
    # persist > 0: persistent workgroups; 600 envs over 16 maps make chunks
    # of tiles that cross map boundaries.  th: threads per workgroup.
    for te, ra, gr, rs, wk, pe, th in [
            (4, 48, 4, 0, 0, 0, 256), (8, 32, 2, 0, 0, 0, 256), (16, 56, 8, 0, 0, 0, 256),
            (4, 0, 1, 0, 0, 0, 256), (8, 63, 64, 0, 0, 0, 256), (4, 40, 8, 256, 0, 0, 256),
            (16, 48, 4, 600, 0, 0, 256), (1, 48, 8, 0, 0, 0, 256), (2, 40, 8, 0, 0, 0, 256),
            (1, 32, 16, 256, 0, 0, 256), (4, 48, 4, 0, 1, 0, 256), (1, 40, 2, 0, 1, 0, 256),
            (16, 0, 1, 256, 1, 0, 256), (8, 63, 64, 0, 1, 0, 256),
            (4, 48, 4, 0, 0, 1, 256), (4, 56, 8, 0, 0, 3, 256), (1, 48, 8, 0, 0, 8, 256),
            (8, 32, 2, 256, 0, 2, 256), (16, 48, 4, 0, 1, 64, 256), (2, 40, 8, 0, 0, 5, 256),
            (4, 56, 8, 0, 0, 0, 512), (16, 56, 8, 0, 0, 0, 1024), (1, 48, 4, 0, 0, 0, 1024),
            (8, 32, 2, 256, 0, 0, 512), (2, 48, 8, 0, 1, 0, 512), (16, 48, 4, 0, 0, 2, 1024),
            (8, 0, 1, 4096, 0, 0, 1024), (4, 56, 8, 0, 2, 0, 256), (1, 0, 1, 256, 2, 0, 256),
            (16, 48, 4, 0, 2, 0, 1024), (8, 63, 64, 0, 2, 3, 512), (2, 32, 2, 512, 2, 0, 256),
            (4, 56, 8, 0, 3, 0, 256), (1, 0, 1, 0, 3, 0, 256), (16, 48, 4, 0, 3, 2, 1024),
            (8, 63, 64, 0, 4, 0, 512), (4, 56, 8, 0, 4, 0, 256), (2, 32, 2, 0, 4, 5, 256),
            (32, 40, 8, 0, 4, 0, 512), (32, 32, 16, 0, 3, 0, 1024), (32, 48, 8, 0, 0, 3, 512),
            (4, 56, 8, 0, 5, 0, 256), (1, 0, 1, 0, 5, 0, 256), (16, 48, 4, 0, 5, 2, 1024),
            (8, 63, 64, 0, 5, 0, 512), (32, 40, 8, 0, 5, 0, 512), (2, 32, 2, 0, 5, 5, 256)]:
        sim = NavSim(w["cfg"], w["maps"], w["res"], w["env_map"], device=0)
        bal = int(th == 1024 or te == 32)  # the larger workgroups also with balanced tiles
        sim.set_tuning(te, ra, gr, rs, wk, pe, th, bal)
        assert sim.get_tuning() == {"tile_envs": te, "refill_at": ra, "groups": gr,
                                    "ray_slots": rs, "walk": wk, "persist": pe, "threads": th,
                                    "balance": bal}
        sim.reset()
        outs = []
        for t in range(3):
            g, st = gpu_step(sim, acts[t], NAVSIM_KERNEL_FUSED)
            outs.append((g, st))
        if ref_out is None:
            ref_out = outs
        else:
            for (ga, sa), (gb, sb) in zip(ref_out, outs):
                for k in ga:
                    assert np.array_equal(ga[k], gb[k]) or k == "final_obs", (te, ra, gr, rs, wk,
                                                                               pe, th, k)
                for k in oracle.STATE_KEYS:
                    assert np.array_equal(sa[k], sb[k]), (te, ra, gr, rs, wk, pe, th, k)
        sim.close()


@pytest.mark.parametrize("wl", ["c2", "c4"])
def test_pooled_obs_same_with_and_without_per_ray_outputs(wl):
    # the step with and without the per-ray debug outputs (ranges, hits,
    # visits) must produce the same observations, rewards, flags and state
    say(f"{wl}: plain steps == steps with per-ray outputs (bitwise), walks 0, 3, 4, 5")
    w = configs.build_workload(wl)
    N = w["cfg"]["num_envs"]
    acts = torch.from_numpy(configs.uniform_actions(3, N, seed=17)).cuda()
    for wk, te, th in [(0, 4, 256), (3, 4, 256), (4, 16, 1024), (5, 16, 512)]:
        sim = NavSim(w["cfg"], w["maps"], w["res"], w["env_map"], device=0, profiles=w["profiles"])
        try:
            sim.set_tuning(te, 48, 8, walk=wk, threads=th)
        except navsim.NavsimError:
            assert wl == "c4" and wk == 4  # 512^2 maps: the byte copy does not fit
            sim.close()
            continue
        sim.reset()
        for t in range(3):
            s0 = sim.get_state()
            o, r, te_, tr, info = sim.step(acts[t])
            got = [x.cpu().numpy().copy() for x in (o, r, te_, tr, info["final_obs"])]
            s1 = sim.get_state()
            sim.set_state(s0)
            sim.step_debug(acts[t])
            torch.cuda.synchronize()
            want = [x.cpu().numpy().copy() for x in (sim.obs, sim.reward, sim.terminated,
                                                      sim.truncated, sim.final_obs)]
            done = (got[2] | got[3]).astype(bool)
            for i, (a, b) in enumerate(zip(got, want)):
                if i == 4:
                    a, b = a[done], b[done]
                assert np.array_equal(a, b), (wk, t, i)
            s2 = sim.get_state()
            assert all(np.array_equal(s1[k], s2[k]) for k in oracle.STATE_KEYS)
        sim.close()


@pytest.mark.parametrize("kname", ["fused", "plain"])
def test_go2_rectangle_on_fine_grid(kname):
    say(f"go2 preset (0.80 x 0.41 m rectangle, 1080 beams, r_max 20 m) on 1 cm rooms maps "
        f"600^2: footprint window of 91 cells per side, kernel={kname}, 3 steps")
    cfg = configs.go2(num_envs=256)
    maps = [configs._maps.gen_rooms_map(7000 + k, w=600, h=600, res=0.01) for k in range(2)]
    res = [0.01, 0.01]
    env_map = configs.contiguous_env_map(256, 2)
    sim, ref = make_pair(cfg, maps, res, env_map)
    tot = run_teacher_forced(sim, ref, 3, KERNELS[kname], label=f"go2-1cm/{kname}")
    assert tot["rays"] > 0
    sim.close()


def test_footprint_window_beyond_limit_is_rejected():
    say("go2 rectangle on 5 mm cells: window of 181 cells, rejected at load")
    cfg = configs.go2(num_envs=4)
    maps = [configs._maps.gen_rooms_map(7000, w=400, h=400, res=0.005)]
    with pytest.raises(navsim.NavsimError) as ei:
        NavSim(cfg, maps, [0.005], np.zeros(4, np.int32), device=0)
    assert ei.value.status == -7
    assert "window" in str(ei.value)
