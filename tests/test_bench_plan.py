"""Host-side checks of bench.py's leg planning: every leg of the benchmark
reads only action rows that exist, for the round-end command
(--steps 20 --warmup 5) and for the defaults."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("steps,warmup,plain,march", [
    (20, 5, 50, 20), (1000, 20, 50, 200), (1, 0, 0, 0), (3, 2, 50, 3), (64, 10, 0, 64)])
def test_every_leg_reads_existing_rows(steps, warmup, plain, march):
    p = bench.plan_legs(steps, warmup, plain, march, 5 if march else 0)
    rows = p["rows"]
    for name, (a, b) in p["legs"].items():
        assert 0 <= a <= b <= rows, name
    assert p["legs"]["timed"] == (warmup, warmup + steps)
    assert p["legs"]["replay"] == p["legs"]["timed"]
    assert p["legs"]["plain"][1] - p["legs"]["plain"][0] == plain
    assert p["legs"]["march"][1] - p["legs"]["march"][0] == march
    # the longest leg sets the row count
    assert rows == warmup + max(steps, plain, march, 5 if march else 0)


def test_round_end_command_plan():
    # python bench.py --gpus 1 --steps 20 --warmup 5: plain leg of 50 steps and
    # a march leg of min(steps, 200) steps need 55 rows
    p = bench.plan_legs(20, 5, 50, min(20, 200), 5)
    assert p["rows"] == 55


def test_bad_counts_rejected():
    with pytest.raises(ValueError):
        bench.plan_legs(0, 5, 50, 20)
    with pytest.raises(ValueError):
        bench.plan_legs(10, -1, 50, 20)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
