"""Pins for the oracle's footprint collision test (section 2.2.1 bitmap
collision, out-of-bounds = occupied; section 2.2.3 collision event).

A disc collides when an occupied cell lies strictly closer than its radius; a
rectangle collides when its interior overlaps an occupied cell's interior.
The oracle restricts the search to candidate cells and uses a separating-axis
test; the brute force here visits every cell (plus a ring outside the map)
and, for the rectangle, clips the rectangle polygon against each cell and
looks at the overlap area.
"""
import math

import numpy as np
import pytest

import oracle


def _s(v):
    return float(np.float32(v))


def brute_disc(occ, s, x, y, r):
    H, W = occ.shape
    for j in range(-3, H + 3):
        for i in range(-3, W + 3):
            filled = not (0 <= i < W and 0 <= j < H) or occ[j, i]
            if not filled:
                continue
            gx = max(i * s - x, 0.0, x - (i + 1) * s)
            gy = max(j * s - y, 0.0, y - (j + 1) * s)
            if math.hypot(gx, gy) < r:
                return True
    return False


def _clip(poly, a, b, c):
    """Keep the part of polygon with a*x + b*y <= c (Sutherland-Hodgman)."""
    out = []
    n = len(poly)
    for k in range(n):
        p, q = poly[k], poly[(k + 1) % n]
        fp, fq = a * p[0] + b * p[1] - c, a * q[0] + b * q[1] - c
        if fp <= 0:
            out.append(p)
        if (fp < 0 < fq) or (fq < 0 < fp):
            t = fp / (fp - fq)
            out.append((p[0] + t * (q[0] - p[0]), p[1] + t * (q[1] - p[1])))
    return out


def _area(poly):
    if len(poly) < 3:
        return 0.0
    return 0.5 * abs(sum(poly[k][0] * poly[(k + 1) % len(poly)][1]
                         - poly[(k + 1) % len(poly)][0] * poly[k][1] for k in range(len(poly))))


def brute_rect(occ, s, x, y, th, L, B):
    """Returns (collides, ambiguous): the largest clipped overlap area decides;
    areas within 1e-10 of zero are reported as ambiguous."""
    H, W = occ.shape
    c, sn = math.cos(th), math.sin(th)
    hl, hb = L / 2, B / 2
    rect = [(x + ux * hl * c - wy * hb * sn, y + ux * hl * sn + wy * hb * c)
            for ux, wy in ((1, 1), (-1, 1), (-1, -1), (1, -1))]
    best = 0.0
    for j in range(-3, H + 3):
        for i in range(-3, W + 3):
            filled = not (0 <= i < W and 0 <= j < H) or occ[j, i]
            if not filled:
                continue
            p = _clip(rect, 1, 0, (i + 1) * s)
            p = _clip(p, -1, 0, -i * s) if p else p
            p = _clip(p, 0, 1, (j + 1) * s) if p else p
            p = _clip(p, 0, -1, -j * s) if p else p
            best = max(best, _area(p) if p else 0.0)
    return best > 1e-10, 0.0 < best <= 1e-10


@pytest.mark.parametrize("seed", range(6))
def test_disc_matches_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    H, W = int(rng.integers(5, 12)), int(rng.integers(5, 12))
    s = _s(rng.choice([0.05, 0.1]))
    occ = (rng.random((H, W)) < 0.2).astype(np.uint8)
    M = oracle.OracleMaps([occ], [s])
    for _ in range(300):
        x, y = rng.uniform(-0.1, W * s + 0.1), rng.uniform(-0.1, H * s + 0.1)
        r = _s(rng.uniform(0.02, 0.3))
        assert M.disc_hits(0, x, y, r) == brute_disc(occ, s, x, y, r)


@pytest.mark.parametrize("seed", range(6))
def test_rect_matches_polygon_clipping(seed):
    rng = np.random.default_rng(200 + seed)
    H, W = int(rng.integers(6, 12)), int(rng.integers(6, 12))
    s = _s(rng.choice([0.05, 0.1]))
    occ = (rng.random((H, W)) < 0.15).astype(np.uint8)
    M = oracle.OracleMaps([occ], [s])
    L, B = _s(0.7), _s(0.31)
    n = 0
    for _ in range(150):
        x, y = rng.uniform(0, W * s), rng.uniform(0, H * s)
        th = _s(rng.uniform(-math.pi, math.pi))
        want, amb = brute_rect(occ, s, x, y, th, L, B)
        if amb:
            continue
        assert M.rect_hits(0, x, y, th, L, B) == want, (x, y, th)
        n += 1
    assert n > 140


def test_disc_tangent_to_wall():
    s = _s(0.05)
    occ = np.zeros((40, 40), np.uint8)
    occ[:, 30] = 1  # wall face at x = 30 s
    M = oracle.OracleMaps([occ], [s])
    r = _s(0.18)
    assert not M.disc_hits(0, 30 * s - r - 1e-3, 1.0, r)
    assert M.disc_hits(0, 30 * s - r + 1e-3, 1.0, r)
    assert not M.disc_hits(0, 1.0, 1.0, r)          # free space
    assert M.disc_hits(0, 30.5 * s, 1.0, r)         # centre inside the wall


def test_out_of_bounds_counts_as_occupied():
    s = _s(0.1)
    occ = np.zeros((10, 10), np.uint8)              # no border
    M = oracle.OracleMaps([occ], [s])
    r = _s(0.2)
    assert not M.disc_hits(0, 0.5, 0.5, r)
    assert M.disc_hits(0, 0.15, 0.5, r)             # reaches x < 0
    assert M.disc_hits(0, 0.5, 0.85, r)             # reaches y > H s
    assert M.rect_hits(0, 0.3, 0.5, 0.0, _s(0.7), _s(0.31))


def test_rect_axis_aligned_interval_form():
    # At heading 0 the rectangle is [x -+ L/2] x [y -+ B/2]; it collides iff an
    # occupied cell's open box meets that open box.
    rng = np.random.default_rng(5)
    s = _s(0.05)
    occ = (rng.random((30, 30)) < 0.05).astype(np.uint8)
    M = oracle.OracleMaps([occ], [s])
    L, B = _s(0.7), _s(0.31)
    for _ in range(300):
        x, y = rng.uniform(0.4, 1.1), rng.uniform(0.2, 1.3)
        want = False
        for j in range(30):
            for i in range(30):
                if occ[j, i] and (x - L / 2 < (i + 1) * s and i * s < x + L / 2
                                  and y - B / 2 < (j + 1) * s and j * s < y + B / 2):
                    want = True
        assert M.rect_hits(0, x, y, 0.0, L, B) == want


def test_free_list_cells_are_clear():
    rng = np.random.default_rng(9)
    s = _s(0.05)
    occ = (rng.random((30, 40)) < 0.03).astype(np.uint8)
    M = oracle.OracleMaps([occ], [s], circumradius=0.12)
    cells = M.free_cells[:M.free_cnt[0]]
    assert len(cells) > 0
    W = 40
    listed = set(int(c) for c in cells)
    for j in range(30):
        for i in range(40):
            cx, cy = _s((i + 0.5) * s), _s((j + 0.5) * s)
            clear = not brute_disc(occ, s, cx, cy, 0.12)
            assert clear == ((j * W + i) in listed)
    assert list(cells) == sorted(cells)
