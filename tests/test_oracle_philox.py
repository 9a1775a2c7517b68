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
