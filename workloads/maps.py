"""Seeded synthetic occupancy maps for the navigation workloads.

This module only draws input data: it places obstacles on a byte grid and
holds none of the simulator's arithmetic (no kinematics, ray casting,
collision or reward).  Both the GPU path and the CPU oracle consume the byte
arrays it returns, so the two sides always see the same maps.

Grid convention (the paper's bitmap state, section 2.2.1): a map is a
``uint8`` array of shape ``(H, W)``; element ``[iy, ix]`` is the cell that
covers ``[ix*s, (ix+1)*s) x [iy*s, (iy+1)*s)`` in world metres, 1 = occupied.
Row index grows with world y; there is no image flip.

The paper trains on two hand-made floor plans (10 x 10 m and 13.5 x 13.5 m,
appendix B, tables 8-9) that are not available; the generators below stand in
for them with the shapes, sizes and occupancy of the workloads this project
measures.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "add_border",
    "rasterise_disc",
    "gen_rect_map",
    "gen_rect_disc_map",
    "gen_rooms_map",
    "gen_uneven_maps",
]


def add_border(occ: np.ndarray, width: int = 1) -> np.ndarray:
    """Mark a solid frame of ``width`` cells around the map as occupied."""
    occ[:width, :] = 1
    occ[-width:, :] = 1
    occ[:, :width] = 1
    occ[:, -width:] = 1
    return occ


def rasterise_disc(occ: np.ndarray, cx: float, cy: float, radius: float, res: float) -> None:
    """Set every cell whose centre lies within ``radius`` metres of (cx, cy)."""
    h, w = occ.shape
    i0 = max(int(np.floor((cx - radius) / res)) - 1, 0)
    i1 = min(int(np.floor((cx + radius) / res)) + 1, w - 1)
    j0 = max(int(np.floor((cy - radius) / res)) - 1, 0)
    j1 = min(int(np.floor((cy + radius) / res)) + 1, h - 1)
    if i1 < i0 or j1 < j0:
        return
    ii = np.arange(i0, i1 + 1)
    jj = np.arange(j0, j1 + 1)
    px = (ii + 0.5) * res - cx
    py = (jj + 0.5) * res - cy
    inside = (py[:, None] ** 2 + px[None, :] ** 2) <= radius * radius
    occ[j0:j1 + 1, i0:i1 + 1] |= inside.astype(np.uint8)


def _interior_fraction(occ: np.ndarray, border: int) -> float:
    inner = occ[border:-border, border:-border]
    return float(inner.mean())


def gen_rect_map(seed: int, w: int = 64, h: int = 64, side_lo: int = 1, side_hi: int = 8,
                 occupancy: float = 0.10) -> np.ndarray:
    """Solid 1-cell border plus axis-aligned rectangles (sides U{lo..hi} cells)
    placed uniformly inside until the interior occupancy reaches ``occupancy``."""
    rng = np.random.default_rng(seed)
    occ = add_border(np.zeros((h, w), dtype=np.uint8))
    while _interior_fraction(occ, 1) < occupancy:
        rw = int(rng.integers(side_lo, side_hi + 1))
        rh = int(rng.integers(side_lo, side_hi + 1))
        x0 = int(rng.integers(1, w - 1 - rw + 1))
        y0 = int(rng.integers(1, h - 1 - rh + 1))
        occ[y0:y0 + rh, x0:x0 + rw] = 1
    return occ


def gen_rect_disc_map(seed: int, w: int = 128, h: int = 128, res: float = 0.05,
                      side_lo: int = 2, side_hi: int = 16, r_lo: float = 0.1, r_hi: float = 0.5,
                      occupancy: float = 0.15) -> np.ndarray:
    """Border plus rectangles and rasterised discs in equal numbers (alternating)
    until the interior occupancy reaches ``occupancy``."""
    rng = np.random.default_rng(seed)
    occ = add_border(np.zeros((h, w), dtype=np.uint8))
    k = 0
    while _interior_fraction(occ, 1) < occupancy:
        if k % 2 == 0:
            rw = int(rng.integers(side_lo, side_hi + 1))
            rh = int(rng.integers(side_lo, side_hi + 1))
            x0 = int(rng.integers(1, w - 1 - rw + 1))
            y0 = int(rng.integers(1, h - 1 - rh + 1))
            occ[y0:y0 + rh, x0:x0 + rw] = 1
        else:
            rad = float(rng.uniform(r_lo, r_hi))
            cx = float(rng.uniform(res, (w - 1) * res))
            cy = float(rng.uniform(res, (h - 1) * res))
            rasterise_disc(occ, cx, cy, rad, res)
        k += 1
    return occ


def _split_rooms(occ, rng, x0, y0, x1, y1, min_side, wall, door):
    """Recursively partition the free box [x0,x1) x [y0,y1) (cells) by walls
    of ``wall`` cells with one door gap of ``door`` cells each."""
    bw, bh = x1 - x0, y1 - y0
    can_v = bw >= 2 * min_side + wall
    can_h = bh >= 2 * min_side + wall
    if not (can_v or can_h):
        return
    # stop early now and then so room sizes vary
    if rng.random() < 0.15 and (bw < 4 * min_side and bh < 4 * min_side):
        return
    vertical = can_v and (not can_h or bw >= bh)
    if vertical:
        xs = int(rng.integers(x0 + min_side, x1 - min_side - wall + 1))
        occ[y0:y1, xs:xs + wall] = 1
        if bh > door:
            d0 = int(rng.integers(y0, y1 - door + 1))
            occ[d0:d0 + door, xs:xs + wall] = 0
        _split_rooms(occ, rng, x0, y0, xs, y1, min_side, wall, door)
        _split_rooms(occ, rng, xs + wall, y0, x1, y1, min_side, wall, door)
    else:
        ys = int(rng.integers(y0 + min_side, y1 - min_side - wall + 1))
        occ[ys:ys + wall, x0:x1] = 1
        if bw > door:
            d0 = int(rng.integers(x0, x1 - door + 1))
            occ[ys:ys + wall, d0:d0 + door] = 0
        _split_rooms(occ, rng, x0, y0, x1, ys, min_side, wall, door)
        _split_rooms(occ, rng, x0, ys + wall, x1, y1, min_side, wall, door)


def gen_rooms_map(seed: int, w: int = 256, h: int = 256, res: float = 0.05,
                  min_room_m: float = 2.0, wall_cells: int = 2, door_m: float = 1.0,
                  n_disc_max: int = 30, r_lo: float = 0.1, r_hi: float = 0.4) -> np.ndarray:
    """Rooms and corridors from a random recursive rectangle partition (2-cell
    walls, one door gap of ``door_m`` per wall, wider than a 0.70 x 0.31 m
    footprint's diagonal) plus U{0..n_disc_max} rasterised discs centred in
    free cells."""
    rng = np.random.default_rng(seed)
    occ = add_border(np.zeros((h, w), dtype=np.uint8))
    min_side = int(round(min_room_m / res))
    door = int(round(door_m / res))
    _split_rooms(occ, rng, 1, 1, w - 1, h - 1, min_side, wall_cells, door)
    n_disc = int(rng.integers(0, n_disc_max + 1))
    placed = 0
    tries = 0
    while placed < n_disc and tries < 100 * (n_disc + 1):
        tries += 1
        i = int(rng.integers(1, w - 1))
        j = int(rng.integers(1, h - 1))
        if occ[j, i]:
            continue
        rad = float(rng.uniform(r_lo, r_hi))
        rasterise_disc(occ, (i + 0.5) * res, (j + 0.5) * res, rad, res)
        placed += 1
    return occ


def gen_uneven_maps(seed: int, count: int, side_lo: int = 96, side_hi: int = 512,
                    res: float = 0.05) -> list[np.ndarray]:
    """``count`` maps with W and H drawn from U{side_lo..side_hi}; even ids use
    the rectangle+disc generator, odd ids the rooms generator."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        w = int(rng.integers(side_lo, side_hi + 1))
        h = int(rng.integers(side_lo, side_hi + 1))
        if k % 2 == 0:
            out.append(gen_rect_disc_map(1000 + k, w=w, h=h, res=res))
        else:
            out.append(gen_rooms_map(1000 + k, w=w, h=h, res=res))
    return out
