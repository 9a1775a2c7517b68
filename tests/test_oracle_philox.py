"""The reset sampler's counter-based generator (Philox4x32-10) against the
published known-answer vectors, plus basic properties of the draws the reset
protocol uses."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], tuple(v[6:10])))
    return rows


def test_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert oracle.philox4x32_10(ctr, key) == want


def test_counter_words_all_matter_and_uniformity():
    base = oracle.philox4x32_10([5, 7, 0, 0], [11, 13])
    for i in range(4):
        c = [5, 7, 0, 0]
        c[i] += 1
        assert oracle.philox4x32_10(c, [11, 13]) != base
    assert oracle.philox4x32_10([5, 7, 0, 0], [11, 14]) != base
    # (w + 1/2) / 2^32 over 4000 draws: chi-square over 16 bins stays sane
    u = np.array([w for a in range(1000) for w in oracle.philox4x32_10([a, 1, 2, 3], [9, 9])],
                 dtype=np.float64)
    u = (u + 0.5) / 2 ** 32
    assert 0.0 < u.min() and u.max() < 1.0
    hist, _ = np.histogram(u, bins=16, range=(0, 1))
    chi2 = ((hist - 250.0) ** 2 / 250.0).sum()
    assert chi2 < 45.0


def test_rollout_actions_follow_the_counter_layout():
    # stream 4 with counter (env, n mod 2^32, n div 2^32): checked word by word
    # through the KAT-pinned block function, including a step index past 2^32
    from workloads import configs
    cfg = configs.make_config(num_envs=40, num_beams=8, num_sectors=8, fov_rad=6.2832,
                              max_range_m=2.0, dt_s=0.1, footprint=0, radius_m=0.1,
                              v_min=0.0, v_max=0.5, w_min=-1.0, w_max=1.0,
                              seed=0x0123456789ABCDEF)
    occ = np.zeros((20, 20), np.uint8)
    ref = oracle.OracleSim(cfg, [occ], [0.1], np.zeros(40, np.int32))
    key = [0x89ABCDEF, 0x01234567]
    for n in (0, 1, 77, (5 << 32) + 3):
        a = ref.rollout_actions(n)
        for e in (0, 1, 39):
            w = oracle.philox4x32_10([e, n & 0xFFFFFFFF, n >> 32, 4], key)
            want = [np.float32(2.0 * ((w[i] + 0.5) / 2 ** 32) - 1.0) for i in (0, 1)]
            assert a[e, 0] == want[0] and a[e, 1] == want[1], (n, e)
    # a fresh draw per step and env, spread over (-1, 1)
    allv = np.concatenate([ref.rollout_actions(n).ravel() for n in range(200)])
    assert -1.0 < allv.min() and allv.max() < 1.0
    assert abs(allv.mean()) < 0.02
    assert not np.array_equal(ref.rollout_actions(3), ref.rollout_actions(4))
