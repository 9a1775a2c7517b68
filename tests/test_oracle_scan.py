"""Pins for the oracle's range scan (eq. 4-5, section 2.2.2).

The oracle finds each ray's first occupied cell by a grid traversal.  These
tests tie it to things it does not compute itself: closed forms (empty map,
axis-aligned wall, rasterised disc bounds, map boundary), a brute-force
minimum over every cell's slab entry distance (the definition of "first
occupied cell along the ray"), and a fine fixed-step march.
"""
import math

import numpy as np
import pytest

import oracle

EPS = 1e-6


def _maps(occ, res):
    return oracle.OracleMaps([occ], [res])


def brute_first_hit(occ, s, ox, oy, dx, dy, rmax):
    """Definition: smallest entry distance over every occupied cell and the
    region outside the map, by the slab method.  Returns (range, hit)."""
    H, W = occ.shape
    best_t, best = math.inf, None

    def slab(x0, x1, y0, y1):
        tn, tf = -math.inf, math.inf
        for o, d, lo, hi in ((ox, dx, x0, x1), (oy, dy, y0, y1)):
            if d == 0.0:
                if not (lo <= o <= hi):
                    return None
                continue
            a, b = (lo - o) / d, (hi - o) / d
            tn, tf = max(tn, min(a, b)), min(tf, max(a, b))
        if tn <= tf and tf >= 0.0:
            return tn, tf
        return None

    for j in range(H):
        for i in range(W):
            if not occ[j, i]:
                continue
            r = slab(i * s, (i + 1) * s, j * s, (j + 1) * s)
            if r is not None:
                t = max(r[0], 0.0)
                if t < best_t:
                    best_t, best = t, j * W + i
    # leaving the map: exit distance of the map rectangle
    r = slab(0.0, W * s, 0.0, H * s)
    t_exit = r[1] if r is not None else 0.0
    if t_exit < best_t:
        best_t, best = t_exit, -2
    if best_t > rmax:
        return rmax, -1
    return best_t, best


def cells_crossed(occ, s, ox, oy, dx, dy, t_stop):
    """Number of grid cells (map plus a ring outside) whose interior the ray
    crosses at distances in [0, t_stop]: brute force over a window."""
    H, W = occ.shape
    n = 0
    for j in range(-2, H + 2):
        for i in range(-2, W + 2):
            tn, tf = -math.inf, math.inf
            ok = True
            for o, d, lo, hi in ((ox, dx, i * s, (i + 1) * s), (oy, dy, j * s, (j + 1) * s)):
                if d == 0.0:
                    if not (lo < o < hi):
                        ok = False
                    continue
                a, b = (lo - o) / d, (hi - o) / d
                tn, tf = max(tn, min(a, b)), min(tf, max(a, b))
            if ok and tn < tf and tf > 0.0 and tn <= t_stop:
                n += 1
    return n


def test_empty_map_returns_max_range():
    # 200 x 200 cells of 0.05 m, nothing occupied; origin at the centre, r_max
    # 3 m < 5 m to every edge: every beam reports r_max and no hit.
    occ = np.zeros((200, 200), np.uint8)
    M = _maps(occ, 0.05)
    rng = np.random.default_rng(0)
    for _ in range(500):
        ox, oy = 5.0 + rng.uniform(-0.5, 0.5), 5.0 + rng.uniform(-0.5, 0.5)
        a = rng.uniform(-math.pi, math.pi)
        r = M.cast(0, ox, oy, math.cos(a), math.sin(a), 3.0)
        assert r.hit == -1 and r.range == 3.0


def test_map_boundary_distance_closed_form():
    # No border, no obstacle: range = distance to where the ray leaves
    # [0, W s] x [0, H s], hit = -2 (out of bounds counts as occupied).
    occ = np.zeros((40, 60), np.uint8)
    s = float(np.float32(0.1))  # the grid uses the float32 cell size
    M = _maps(occ, s)
    rng = np.random.default_rng(1)
    checked = 0
    for _ in range(400):
        ox, oy = rng.uniform(0.3, 5.7), rng.uniform(0.3, 3.7)
        a = rng.uniform(-math.pi, math.pi)
        dx, dy = math.cos(a), math.sin(a)
        r = M.cast(0, ox, oy, dx, dy, 100.0)
        if r.grazing:
            continue
        tx = ((60 * s - ox) / dx) if dx > 0 else ((0.0 - ox) / dx) if dx < 0 else math.inf
        ty = ((40 * s - oy) / dy) if dy > 0 else ((0.0 - oy) / dy) if dy < 0 else math.inf
        assert r.hit == -2
        assert abs(r.range - min(tx, ty)) < 1e-12
        checked += 1
    assert checked > 300


@pytest.mark.parametrize("side", ["+x", "-x", "+y", "-y"])
def test_axis_aligned_wall_d_over_cos(side):
    # A full-height wall column at perpendicular distance D: a beam at angle
    # beta from the wall normal reads D / cos(beta) and hits the wall cell
    # that contains the end point.
    s = float(np.float32(0.05))
    n = 160
    occ = np.zeros((n, n), np.uint8)
    wall = 120
    if side in ("+x", "-x"):
        occ[:, wall if side == "+x" else n - 1 - wall] = 1
    else:
        occ[wall if side == "+y" else n - 1 - wall, :] = 1
    M = _maps(occ, s)
    rng = np.random.default_rng(2)
    for _ in range(300):
        beta = rng.uniform(-1.2, 1.2)
        u = rng.uniform(2.0, 4.0)
        v = rng.uniform(2.0, 6.0)
        # frame: normal direction towards the wall
        if side == "+x":
            ox, oy = u, v
            dx, dy = math.cos(beta), math.sin(beta)
            D = wall * s - ox
        elif side == "-x":
            ox, oy = n * s - u, v
            dx, dy = -math.cos(beta), math.sin(beta)
            D = ox - (n - 1 - wall + 1) * s
        elif side == "+y":
            ox, oy = v, u
            dx, dy = math.sin(beta), math.cos(beta)
            D = wall * s - oy
        else:
            ox, oy = v, n * s - u
            dx, dy = math.sin(beta), -math.cos(beta)
            D = oy - (n - 1 - wall + 1) * s
        expect = D / math.cos(beta)
        r = M.cast(0, ox, oy, dx, dy, 20.0)
        if r.grazing:
            continue
        ex, ey = ox + expect * dx, oy + expect * dy
        if expect > 20.0 or not (0 < ex < n * s and 0 < ey < n * s):
            continue
        assert abs(r.range - expect) < 1e-9
        if side in ("+x", "-x"):
            assert r.hit % n == (wall if side == "+x" else n - 1 - wall)
            assert r.hit // n == int(math.floor(ey / s))
        else:
            assert r.hit // n == (wall if side == "+y" else n - 1 - wall)
            assert r.hit % n == int(math.floor(ex / s))


def test_rasterised_disc_bounds():
    # Cells whose centre is within R of C are occupied.  The occupied set lies
    # between the discs of radius R - s/sqrt2 and R + s/sqrt2, so a ray aimed
    # at the disc reads between the analytic entry distances of those discs.
    from workloads.maps import rasterise_disc
    s = float(np.float32(0.05))
    occ = np.zeros((200, 200), np.uint8)
    cx, cy, R = 5.02, 4.97, 1.3
    rasterise_disc(occ, cx, cy, R, s)
    M = _maps(occ, s)
    rng = np.random.default_rng(3)

    def t_circle(ox, oy, dx, dy, rho):
        bx, by = cx - ox, cy - oy
        b = bx * dx + by * dy
        c = bx * bx + by * by - rho * rho
        disc = b * b - c
        if disc < 0:
            return None
        return b - math.sqrt(disc)

    n_in = 0
    for _ in range(400):
        ang = rng.uniform(-math.pi, math.pi)
        dist = rng.uniform(2.0, 3.5)
        ox, oy = cx + dist * math.cos(ang), cy + dist * math.sin(ang)
        aim = math.atan2(cy - oy, cx - ox) + rng.uniform(-0.3, 0.3)
        dx, dy = math.cos(aim), math.sin(aim)
        r = M.cast(0, ox, oy, dx, dy, 10.0)
        lo = t_circle(ox, oy, dx, dy, R + s / math.sqrt(2))
        hi = t_circle(ox, oy, dx, dy, R - s / math.sqrt(2))
        if lo is None:
            continue
        assert r.hit >= 0
        assert r.range >= lo - 1e-12
        if hi is not None:
            assert r.range <= hi + 1e-12
            n_in += 1
    assert n_in > 300


@pytest.mark.parametrize("seed", [10, 11, 12, 13])
def test_traversal_equals_brute_force_minimum(seed):
    # Tiny random maps: the traversal's hit cell equals the brute-force argmin
    # of slab entry distances and its range agrees to 1e-12, for every
    # non-grazing ray; grazing rays are counted and stay rare.
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(6, 14)), int(rng.integers(6, 14))
    s = float(np.float32(rng.choice([0.05, 0.1, 0.25])))
    occ = (rng.random((H, W)) < 0.25).astype(np.uint8)
    M = _maps(occ, s)
    graze = 0
    n = 0
    for _ in range(400):
        ox, oy = rng.uniform(-0.2 * s, W * s * 1.02), rng.uniform(-0.2 * s, H * s * 1.02)
        a = rng.uniform(-math.pi, math.pi)
        dx, dy = math.cos(a), math.sin(a)
        rmax = float(rng.uniform(0.2, 1.5) * max(W, H) * s)
        r = M.cast(0, ox, oy, dx, dy, rmax)
        if r.grazing:
            graze += 1
            continue
        i, j = math.floor(ox / s), math.floor(oy / s)
        if not (0 <= i < W and 0 <= j < H):
            assert r.hit == -2 and r.range == 0.0
            continue
        if occ[j, i]:
            assert r.hit == j * W + i and r.range == 0.0
            continue
        rb, hb = brute_first_hit(occ, s, ox, oy, dx, dy, rmax)
        assert r.hit == hb, (ox, oy, a, rmax)
        assert abs(r.range - rb) < 1e-12
        # visits = cells crossed up to the stopping distance
        stop = r.range if r.hit != -1 else rmax
        assert r.visits == cells_crossed(occ, s, ox, oy, dx, dy, stop)
        n += 1
    assert n > 180 and graze < 20


def test_traversal_vs_fine_step_march():
    # A fixed-step march with h = s/1000 lands within h of the traversal's
    # range and on the same cell, except for rays passing within 2h of a
    # corner (where the march may skip a clipped cell).
    rng = np.random.default_rng(20)
    H, W, s = 24, 30, float(np.float32(0.05))
    occ = (rng.random((H, W)) < 0.12).astype(np.uint8)
    M = _maps(occ, s)
    h = s / 1000
    n = 0
    for _ in range(300):
        ox, oy = rng.uniform(0.01, W * s - 0.01), rng.uniform(0.01, H * s - 0.01)
        if occ[int(oy / s), int(ox / s)]:
            continue
        a = rng.uniform(-math.pi, math.pi)
        dx, dy = math.cos(a), math.sin(a)
        r = M.cast(0, ox, oy, dx, dy, 1.0)
        if r.grazing or r.perp < 2 * h or abs(r.t_end - 1.0) < 2 * h:
            continue
        rm, hm = M.march(0, ox, oy, dx, dy, 1.0, h)
        assert hm == r.hit
        assert r.range - 1e-12 <= rm <= r.range + h + 1e-12
        n += 1
    assert n > 200


def test_origin_in_occupied_or_outside():
    occ = np.zeros((10, 10), np.uint8)
    occ[4, 5] = 1
    M = _maps(occ, 0.1)
    r = M.cast(0, 0.55, 0.45, 1.0, 0.0, 3.0)
    assert r.range == 0.0 and r.hit == 4 * 10 + 5
    r = M.cast(0, -0.05, 0.45, 1.0, 0.0, 3.0)
    assert r.range == 0.0 and r.hit == -2


def test_beam_angles_full_circle_and_fov():
    sim_cfg = dict(num_envs=1, num_beams=8, num_sectors=8, fov_rad=2 * math.pi, max_range_m=1,
                   dt_s=0.1, horizon=200, goal_radius_m=0.2, c_progress=2, r_success=10,
                   r_collision=-10, footprint=0, radius_m=0.1, length_m=0, width_m=0, v_min=0,
                   v_max=1, w_min=-1, w_max=1, goal_min_dist_m=0.5, reset_max_tries=8, seed=1)
    occ = np.zeros((20, 20), np.uint8)
    sim = oracle.OracleSim(sim_cfg, [occ], [0.1], np.zeros(1, np.int32))
    got = [sim.beam_angle(k) for k in range(8)]
    assert np.allclose(got, [-math.pi + k * math.pi / 4 for k in range(8)], atol=1e-15)
    sim_cfg.update(fov_rad=math.radians(270.0), num_beams=5, num_sectors=5)
    sim = oracle.OracleSim(sim_cfg, [occ], [0.1], np.zeros(1, np.int32))
    got = [sim.beam_angle(k) for k in range(5)]
    fov = float(np.float32(math.radians(270.0)))
    assert abs(got[0] + fov / 2) < 1e-15 and abs(got[-1] - fov / 2) < 1e-12


def test_march_at_the_paper_step_closed_forms():
    # h = 0.03 m on 0.05 m cells: samples are closer than a cell, so an
    # axis-aligned ray cannot step over a cell: it stops at the first sample
    # past the wall's entry distance, range in [d, d + h), same cell
    s = float(np.float32(0.05))
    occ = np.zeros((40, 40), np.uint8)
    occ[:, 30] = 1
    M = _maps(occ, s)
    h = 0.03
    for ox in (0.101, 0.4, 0.77, 1.2345):
        oy = 0.9
        r = M.cast(0, ox, oy, 1.0, 0.0, 5.0)
        rm, hm = M.march(0, ox, oy, 1.0, 0.0, 5.0, h)
        assert hm == r.hit == int(oy / s) * 40 + 30
        assert r.range <= rm < r.range + h
        k = rm / h
        assert abs(k - round(k)) < 1e-9  # range is a whole number of steps
    # beyond r_max: the largest sample not past r_max decides, range = r_max
    rm, hm = M.march(0, 0.1, 0.9, 1.0, 0.0, 0.5, h)
    assert (rm, hm) == (0.5, -1)
    # origin out of bounds: sample 0 is outside, range 0, hit -2
    assert M.march(0, -0.01, 0.9, 1.0, 0.0, 5.0, h) == (0.0, -2)


def test_march_scan_mode_step_pools_the_marched_beams():
    # a step in scan mode 1 observes the per-sector minima of orc_march ranges
    from workloads import configs, maps as gm
    occ = gm.gen_rect_disc_map(4, w=70, h=60, res=0.05)
    cfg = configs.make_config(num_envs=10, num_beams=60, num_sectors=6, fov_rad=2 * math.pi,
                              max_range_m=2.5, dt_s=0.1, footprint=0, radius_m=0.18,
                              v_min=0.0, v_max=0.5, w_min=-1.0, w_max=1.0)
    cfg.update(scan_mode=1, march_step_m=0.03)
    sim = oracle.OracleSim(cfg, [occ], [0.05], np.zeros(10, np.int32))
    sim.reset()
    out = sim.step(np.zeros((10, 2), np.float32))
    st = sim.state
    for e in range(10):
        if out["reset"][e]:
            continue
        want = []
        for k in range(60):
            a = float(st["th"][e]) + sim.beam_angle(k)
            rg, _ = sim.maps.march(0, float(st["x"][e]), float(st["y"][e]), math.cos(a),
                                   math.sin(a), float(np.float32(2.5)), float(np.float32(0.03)))
            want.append(np.float32(rg))
        want = np.array(want).reshape(6, 10).min(axis=1)
        assert np.array_equal(out["obs"][e, :6], want), e


@pytest.mark.parametrize("seed", [3, 4])
def test_cells_walked_bound_the_range_from_below(seed):
    # Within distance t a ray crosses at most t |dx| / s + 1 vertical and
    # t |dy| / s + 1 horizontal grid lines, so the cell it enters after k
    # steps of the traversal is at least (k - 2) s / (|dx| + |dy|) away:
    # a relation between the oracle's ranges and visit counts (visits =
    # k + 1) that neither computes from the other, every ray, grazing or not.
    rng = np.random.default_rng(seed)
    worst = math.inf
    for _ in range(6):
        H, W = int(rng.integers(8, 40)), int(rng.integers(8, 40))
        s = float(np.float32(rng.choice([0.05, 0.1])))
        occ = (rng.random((H, W)) < rng.uniform(0.02, 0.3)).astype(np.uint8)
        M = _maps(occ, s)
        for _ in range(300):
            ox, oy = rng.uniform(0.0, W * s), rng.uniform(0.0, H * s)
            a = rng.uniform(-math.pi, math.pi)
            dx, dy = math.cos(a), math.sin(a)
            rmax = float(rng.uniform(0.3, 1.2) * max(W, H) * s)
            r = M.cast(0, ox, oy, dx, dy, rmax)
            if r.hit == -1 or r.range == 0.0:
                continue
            k = r.visits - 1
            bound = (k - 2) * s / (abs(dx) + abs(dy))
            assert r.range >= bound - 1e-12, (ox, oy, a, k, r.range, bound)
            worst = min(worst, r.range - bound)
    assert worst < 2.5 * 0.1  # the bound is not vacuous: it comes within a few cells
