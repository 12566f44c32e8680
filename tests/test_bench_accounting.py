"""Host logic of bench.py: the per-kernel algorithmic byte counts from a
per-level record, the whole-BFS byte count, the averaging, and the one-GPU
contract (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def lvl(mark, frontier, edges, pc=0, pe=0):
    return {"mark": mark, "frontier": frontier, "edges": edges,
            "pull_candidates": pc, "pull_edges": pe}


# a hand-made search: claim, claim with touch marks, push mark, pull, then
# the empty level that ends it
LEVELS = [
    lvl(0, 1, 10),
    lvl(3, 10, 1000),
    lvl(1, 500, 100000, pc=2000, pe=9000),
    lvl(2, 2000, 50000, pc=30000, pe=45000),
    lvl(0, 700, 800),
    lvl(0, 0, 0),
]


def test_claim_bytes_by_level_kind():
    hot = 1000
    want = (4.125 * 10 + 20 * 1 + 53 * 10          # claim level, 10 vertices claimed
            + 4.125 * 1000 + 20 * 10 + 9 * 500     # touch-mark claim level
            + 36 * hot + 36 * hot                   # mark levels: the bitmap build
            + 4.125 * 800 + 20 * 700 + 0)          # last claim level, nothing new
    assert bench.claim_bytes(LEVELS, hot) == pytest.approx(want)


def test_mark_expand_bytes_count_push_levels_and_their_resolve():
    want = 4.125 * 100000 + 16 * 500 + 1 * 2000 + 44 * 2000 + 4.125 * 9000
    assert bench.mark_expand_bytes(LEVELS) == pytest.approx(want)


def test_pull_bytes_count_pull_levels_only():
    n_active = 1 << 20
    want = n_active / 8 + 8 * 30000 + 4.125 * 45000 + 13 * 700
    assert bench.pull_bytes(LEVELS, n_active) == pytest.approx(want)


def test_whole_bfs_bytes_formula():
    n, a, r = 1 << 22, 10 ** 8, 2 * 10 ** 6
    assert bench.bfs_bytes(n, a, r) == pytest.approx(4 * a + a / 8 + 24 * r + 8 * n + n / 4)


def test_harmonic_mean_and_percentile():
    assert bench.harmonic([1.0, 2.0, 4.0]) == pytest.approx(3 / (1 + 0.5 + 0.25))
    assert bench.harmonic([]) == 0.0
    assert bench.harmonic([0.0, 2.0]) == pytest.approx(2.0)   # failed roots drop out
    assert bench.pct([1.0, 2.0, 3.0, 4.0, 5.0], 50) == 3.0


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""
