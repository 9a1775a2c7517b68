"""Pins of the reset-proposal oracle (geodesic distance, difficulty bins,
labelled pairs, rejection sampler, exact proposal check, pooled input): closed
forms on empty and hand-built maps, an independent shortest-path routine, and
brute force on small maps."""
import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
from oracle import geodesic as G


def grid_graph_hops(cfree: np.ndarray, a: int) -> np.ndarray:
    """Unweighted shortest paths with scipy over the 4-neighbour graph of
    C-free cells (an independent routine); -1 = unreachable."""
    H, W = cfree.shape
    idx = np.arange(W * H).reshape(H, W)
    rows, cols = [], []
    f = cfree.astype(bool)
    for di, dj in ((0, 1), (1, 0)):
        a_ = idx[:H - di, :W - dj][f[:H - di, :W - dj] & f[di:, dj:]]
        b_ = idx[di:, dj:][f[:H - di, :W - dj] & f[di:, dj:]]
        rows += [a_, b_]
        cols += [b_, a_]
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    g = csr_matrix((np.ones(len(r)), (r, c)), shape=(W * H, W * H))
    d = shortest_path(g, method="D", unweighted=True, indices=a)
    out = np.where(np.isinf(d), -1, d).astype(np.int64)
    if not f.ravel()[a]:
        out[:] = -1
    return out.reshape(H, W)


def test_empty_grid_gives_manhattan_distance():
    cf = np.ones((23, 31), np.uint8)
    a = 7 * 31 + 11
    f = G.bfs_field(cf, a, 10_000)
    jj, ii = np.mgrid[0:23, 0:31]
    assert np.array_equal(f, np.abs(ii - 11) + np.abs(jj - 7))
    # depth cap: cells beyond max_hops are unreached
    f5 = G.bfs_field(cf, a, 5)
    man = np.abs(ii - 11) + np.abs(jj - 7)
    assert np.array_equal(f5, np.where(man <= 5, man, -1))


def test_wall_with_one_gap():
    # a vertical wall at column 10 with a single gap at row 0: from (2, 5) to
    # (18, 5) the path goes up to row 0, through, and back down
    cf = np.ones((12, 21), np.uint8)
    cf[1:, 10] = 0
    f = G.bfs_field(cf, 5 * 21 + 2, 1000)
    assert f[5, 18] == (10 - 2) + 5 + 5 + (18 - 10)
    assert f[3, 10] == -1  # wall cells are never reached
    # no gap: the other side is unreachable
    cf[0, 10] = 0
    f = G.bfs_field(cf, 5 * 21 + 2, 1000)
    assert (f[:, 11:] == -1).all() and f[5, 9] == 7


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bfs_matches_an_independent_shortest_path_routine(seed):
    rng = np.random.default_rng(seed)
    cf = (rng.random((37, 29)) > 0.3).astype(np.uint8)
    a = int(rng.choice(np.nonzero(cf.ravel())[0]))
    assert np.array_equal(G.bfs_field(cf, a, 100_000), grid_graph_hops(cf, a))
    # a start that is not C-free reaches nothing
    b = int(np.nonzero(cf.ravel() == 0)[0][0])
    assert (G.bfs_field(cf, b, 100) == -1).all()


def test_bin_edges():
    s = float(np.float32(0.05))  # 0.0500000007...: h s is slightly above h / 20
    assert G.bin_of(s, 19, 1.0, 12.0, 8) == -1
    assert G.bin_of(s, 20, 1.0, 12.0, 8) == 0
    # bin width 1.375 m = 27.5 hops: 47 hops = 2.35 m (bin 0), 48 = 2.4 m (bin 1)
    assert G.bin_of(s, 47, 1.0, 12.0, 8) == 0
    assert G.bin_of(s, 48, 1.0, 12.0, 8) == 1
    assert G.bin_of(s, 239, 1.0, 12.0, 8) == 7
    assert G.bin_of(s, 240, 1.0, 12.0, 8) == -1
    assert G.bin_of(s, -1, 1.0, 12.0, 8) == -1
    assert G.max_hops(s, 1.0, 12.0, 8) == 239
    # every hop count in range lands in exactly the bin its distance says
    for h in range(20, 240):
        k = G.bin_of(s, h, 1.0, 12.0, 8)
        assert 1.0 + k * 1.375 <= h * s + 1e-9 and h * s < 1.0 + (k + 1) * 1.375 + 1e-9


def _small_reach(seed=4, W=60, H=50, density=0.25):
    rng = np.random.default_rng(seed)
    cf = (rng.random((H, W)) > density).astype(np.uint8)
    return G.ReachMap(cf, 0.1, seed=0xABCDEF0123, d_lo=0.5, d_hi=4.5, nbins=4, gmd=0.3)


def _picked(w, n):
    return (int(w) * n) >> 32


def test_label_start_is_the_min_key_goal_of_each_bin():
    R = _small_reach()
    key = [int(R.key[0]), int(R.key[1])]
    for sid in (0, 1, 17, 2 ** 31 + 5):
        a, goals, hops = R.label_start(sid)
        w = oracle.philox4x32_10([sid & 0xFFFFFFFF, 0, 0, 6], key)
        assert a == int(R.free[_picked(w[0], len(R.free))])
        field = grid_graph_hops(R.cfree, a).ravel()
        for k in range(R.nbins):
            best = None
            for b in range(R.W * R.H):
                h = int(field[b])
                if h < 0 or h > R.depth or R.bin_of(h) != k:
                    continue
                if R.cell_dist(a, b) < R.gmd:
                    continue
                kk = oracle.philox4x32_10([sid & 0xFFFFFFFF, b, 0, 5], key)[0]
                if best is None or kk < best[0]:
                    best = (kk, b, h)
            if best is None:
                assert goals[k] == -1 and hops[k] == -1
            else:
                assert (goals[k], hops[k]) == (best[1], best[2]), (sid, k)


def test_verify_and_rejection_sampler_by_brute_force():
    R = _small_reach(seed=9)
    key = [int(R.key[0]), int(R.key[1])]
    n = len(R.free)
    for e, ep, k in [(0, 0, 0), (5, 2, 1), (9, 1, 2), (3, 7, 3)]:
        t, a, b, h = R.reject(e, ep, k, 400)
        # replay the attempts by hand
        want = None
        for tt in range(400):
            w = oracle.philox4x32_10([e, ep, tt, 7], key)
            aa, bb = int(R.free[_picked(w[0], n)]), int(R.free[_picked(w[1], n)])
            hh = int(grid_graph_hops(R.cfree, aa).ravel()[bb])
            hh = hh if hh <= R.depth else -1
            if R.cell_dist(aa, bb) >= R.gmd and R.bin_of(hh) == k:
                want = (tt, aa, bb, hh)
                break
        assert want is not None and (t, a, b, h) == want
        assert R.verify(a, b, k) == (True, h)
        assert R.verify(a, b, (k + 1) % R.nbins)[0] is False
    # a blocked endpoint fails the check whatever its distance
    blocked = int(np.nonzero(R.cfree.ravel() == 0)[0][0])
    assert R.verify(blocked, int(R.free[0]), 0)[0] is False
    assert R.verify(int(R.free[0]), blocked, 0)[0] is False


def test_pool32_is_block_max():
    rng = np.random.default_rng(2)
    occ = (rng.random((256, 256)) < 0.01).astype(np.uint8)
    want = occ.reshape(32, 8, 32, 8).max(axis=(1, 3)).astype(np.float32).ravel()
    assert np.array_equal(G.pool32(occ), want)
    occ = (rng.random((70, 100)) < 0.02).astype(np.uint8)  # ragged blocks
    got = G.pool32(occ).reshape(32, 32)
    for q in range(32):
        for p in range(32):
            blk = occ[q * 70 // 32:(q + 1) * 70 // 32, p * 100 // 32:(p + 1) * 100 // 32]
            assert got[q, p] == float(blk.max())


def test_decode_proposal_closed_forms():
    W, H = 40, 30
    assert G.decode_proposal(W, H, [0, 0, 0, 0.9999, 0.9999])[:2] == (0, (H - 1) * W + W - 1)
    a, b, th = G.decode_proposal(W, H, [0.5, 0.5, 0.5, -3.0, 7.0])
    assert a == 15 * W + 20 and b == (H - 1) * W + 0
    assert th == np.float32(0.5 * math.pi)
    a, b, th = G.decode_proposal(W, H, [float("nan"), 0.26, 2.0, 0.1, float("nan")])
    assert a == 7 * W + 0 and b == 0 * W + 4 and th == np.float32(math.pi)


def test_snap_cell_closed_forms():
    cf = np.ones((10, 12), np.uint8)
    R = G.ReachMap(cf, 0.1, seed=1, d_lo=0.2, d_hi=1.0, nbins=2, gmd=0.1)
    assert all(R.snap(c) == c for c in range(120))
    cf = np.zeros((10, 12), np.uint8)
    cf[7, 3] = 1
    R = G.ReachMap(cf, 0.1, seed=1, d_lo=0.2, d_hi=1.0, nbins=2, gmd=0.1)
    assert all(R.snap(c) == 7 * 12 + 3 for c in range(120))
    # two free cells at L1 distance 2 from (5, 5): (5, 3) and (7, 5); the
    # smaller index wins the tie
    cf = np.zeros((10, 12), np.uint8)
    cf[3, 5] = 1
    cf[5, 7] = 1
    R = G.ReachMap(cf, 0.1, seed=1, d_lo=0.2, d_hi=1.0, nbins=2, gmd=0.1)
    assert R.snap(5 * 12 + 5) == 3 * 12 + 5
    assert R.snap(5 * 12 + 6) == 5 * 12 + 7  # distance 1 beats distance 3
    assert G.ReachMap(np.zeros((4, 4), np.uint8), 0.1, seed=1).snap(5) == -1


def test_reset_to_reproduces_a_sampled_reset():
    # resetting to the pose a sampled reset chose gives that reset's state and
    # observation (the same observation, without the sampling)
    from workloads import configs, maps as gm
    occ = gm.gen_rect_disc_map(3, w=80, h=64, res=0.05)
    cfg = configs.make_config(num_envs=12, num_beams=60, num_sectors=6, fov_rad=6.283185307,
                              max_range_m=3.0, dt_s=0.1, footprint=0, radius_m=0.18,
                              v_min=0.0, v_max=0.5, w_min=-1.0, w_max=1.0)
    a = oracle.OracleSim(cfg, [occ], [0.05], np.zeros(12, np.int32))
    obs_a, _ = a.reset()
    st = a.get_state()
    pose = np.stack([st["x"], st["y"], st["th"], st["gx"], st["gy"]], 1)
    b = oracle.OracleSim(cfg, [occ], [0.05], np.zeros(12, np.int32))
    b.reset()
    b.state["ep"][:] = 0
    obs_b = b.reset_to(pose)
    for k in oracle.STATE_KEYS:
        assert np.array_equal(a.state[k], b.state[k]), k
    assert np.array_equal(obs_a, obs_b)
    # masked: untouched rows keep their state
    keep = b.get_state()
    mask = (np.arange(12) % 3 == 0).astype(np.uint8)
    b.reset_to(np.zeros((12, 5), np.float32) + 0.5, mask)
    for k in oracle.STATE_KEYS:
        assert np.array_equal(b.state[k][mask == 0], keep[k][mask == 0]), k
    assert (b.state["x"][mask == 1] == np.float32(0.5)).all()
