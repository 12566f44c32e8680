"""Host logic of bench.py: the per-kernel algorithmic byte counts from a
per-level record, the whole-BFS byte counts, the averaging, and the one-GPU
contract (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def lvl(mark, frontier, edges, pc=0, pe=0, fin=0.0):
    return {"mark": mark, "frontier": frontier, "edges": edges,
            "pull_candidates": pc, "pull_edges": pe, "finish_ms": fin}


# a hand-made search: claim, claim with touch marks, push mark, pull, then
# the empty level that ends it
LEVELS = [
    lvl(0, 1, 10),
    lvl(3, 10, 1000),
    lvl(1, 500, 100000, pc=2000, pe=9000),
    lvl(2, 2000, 50000, pc=30000, pe=145000),
    lvl(0, 700, 800),
    lvl(0, 0, 0),
]


def test_claim_bytes_by_level_kind():
    nwords = 1 << 15          # the whole bitmap, not its LDS-resident prefix
    want = (4.125 * 10 + 20 * 1 + 53 * 10          # claim level, 10 vertices claimed
            + 4.125 * 1000 + 20 * 10 + 16 * 500    # claim-touch level: the atomic min
            + 36 * nwords + 36 * nwords             # mark levels: the level bitmap build
            + 4.125 * 800 + 20 * 700 + 0)          # last claim level, nothing new
    assert bench.claim_bytes(LEVELS, nwords) == pytest.approx(want)


def test_mark_expand_bytes_count_push_levels_and_their_resolve():
    # the resolve's examined adjacencies past the three in the head entry
    want = 4.125 * 100000 + 16 * 500 + 1 * 2000 + 44 * 2000 + 4.125 * (9000 - 3 * 2000)
    assert bench.mark_expand_bytes(LEVELS) == pytest.approx(want)


def test_pull_bytes_count_pull_levels_only():
    n_active = 1 << 20
    want = n_active / 8 + 16 * 30000 + 4.125 * (145000 - 3 * 30000) + 13 * 700
    assert bench.pull_bytes(LEVELS, n_active) == pytest.approx(want)


def test_searches_decided_in_the_head_entry_add_no_row_bytes():
    L = [lvl(2, 100, 1000, pc=50, pe=60), lvl(0, 10, 20)]
    assert bench.pull_bytes(L, 64) == pytest.approx(64 / 8 + 16 * 50 + 13 * 10)


def test_finish_bytes_by_level_kind():
    nwords = 1 << 15
    n = nwords * 32
    want = (12 * 10                                 # claim level: visited bit per new vertex
            # claim-touch level: visited words, the parent words of the
            # vertices not visited before it (root + 10), tags of the words
            # with new vertices
            + 4 * nwords + 8 * (n - 11) + 32 * 500 + 37.125 * 500
            + 32 * nwords + 37.125 * 2000          # push mark level
            + 32 * nwords + 37.125 * 700           # pull level
            + 0)                                   # last claim level reached nothing
    assert bench.finish_bytes(LEVELS, nwords) == pytest.approx(want)
    # a claim level whose new frontier holds n/64 vertices or more rebuilds the bitmap
    big = [lvl(0, 5, 50), lvl(0, nwords * 32 // 64, 10)]
    assert bench.finish_bytes(big, nwords) == pytest.approx(36 * nwords + 12 * 0 +
                                                            bench.finish_bytes(big[1:], nwords))
    # a pull level followed by another pull level builds no queue
    pp = [lvl(2, 100, 5000, pc=10, pe=10), lvl(2, 400, 9000, pc=5, pe=5), lvl(0, 3, 3)]
    assert bench.finish_bytes(pp, nwords) == pytest.approx(
        32 * nwords + 1.125 * 400 + 32 * nwords + 37.125 * 3)


def test_claim_touch_finish_reads_the_parent_words_of_the_unvisited_active_vertices():
    nwords = 1 << 10
    lv = [lvl(0, 1, 40), lvl(0, 40, 3000), lvl(3, 2000, 90000), lvl(0, 5000, 100)]
    seen = 1 + 40 + 2000
    for n_active in (nwords * 32, 20000):
        want = (12 * 40 + 36 * nwords           # claim levels (the second rebuilds the bitmap)
                + 4 * nwords + 8 * (n_active - seen) + 32 * min(nwords, 5000)
                + 37.125 * 5000
                + 0)                           # the last claim level reached nothing
        assert bench.finish_bytes(lv, nwords, n_active) == pytest.approx(want)


def test_examined_bytes_is_the_sum_of_the_kernels_plus_init_and_output():
    n, n_active = 1 << 20, 700000
    nwords = n // 32
    want = (bench.claim_bytes(LEVELS, nwords) + bench.mark_expand_bytes(LEVELS)
            + bench.pull_bytes(LEVELS, n_active) + bench.finish_bytes(LEVELS, nwords, n_active)
            + 8 * n_active + 4 * nwords + 32 * nwords + 20 * n)
    assert bench.examined_bytes(LEVELS, n, n_active) == pytest.approx(want)


def test_whole_bfs_push_bytes_formula():
    n, a, r = 1 << 22, 10 ** 8, 2 * 10 ** 6
    assert bench.bfs_bytes(n, a, r) == pytest.approx(4 * a + a / 8 + 24 * r + 8 * n + n / 4)


class _St:
    def __init__(self, launches, expand, mark, pull, finish=3.0, small=0.25):
        self.expand_launches, self.expand_ms, self.mark_ms, self.pull_ms = \
            launches, expand, mark, pull
        self.finish_ms, self.small_ms = finish, small


def test_device_loop_levels_are_counted_once():
    lv = [lvl(4, 1, 10), lvl(4, 10, 100), lvl(0, 50, 20000), lvl(4, 30, 60), lvl(4, 0, 0)]
    nwords = 1 << 10
    assert bench.small_levels_bytes(lv) == pytest.approx(
        4.125 * 10 + 20 * 1 + 53 * 10 + 4.125 * 100 + 20 * 10 + 53 * 50
        + 4.125 * 60 + 20 * 30 + 0)
    # loop levels add nothing to the level kernels' counts
    assert bench.claim_bytes(lv, nwords) == pytest.approx(4.125 * 20000 + 20 * 50 + 53 * 30)
    assert bench.finish_bytes(lv, nwords) == pytest.approx(12 * 30)


def test_kernel_split_attributes_times_and_bytes():
    lv = [dict(L, finish_ms=0.5) for L in LEVELS]
    st = _St(6, expand=3.0, mark=1.0, pull=0.5)
    n, n_active = 1 << 20, 700000
    sp = bench.kernel_split([st, st], [lv, lv], n, n_active)
    assert sp["k_expand"]["launches"] == 12
    assert sp["k_expand"]["device_ms"] == pytest.approx(2 * 1.5)
    assert sp["k_expand_mark"]["device_ms"] == pytest.approx(2 * 1.5)
    assert sp["k_finish"]["device_ms"] == pytest.approx(2 * 3.0)
    assert sp["k_small_levels"]["device_ms"] == pytest.approx(2 * 0.25)
    b = bench.mark_expand_bytes(lv) + bench.pull_bytes(lv, n_active)
    assert sp["k_expand_mark"]["bytes_per_launch"] == pytest.approx(2 * b / 12, rel=1e-6)
    assert sp["k_expand_mark"]["achieved_gbs"] == pytest.approx(2 * b / 3e-3 / 1e9, abs=0.01)


def test_profiled_traffic_requires_exact_kernel_file_and_current_sources(tmp_path):
    # no summary for an unknown workload
    assert bench.profiled_traffic("k_expand", "no_such_workload") is None


def test_harmonic_mean_and_percentile():
    assert bench.harmonic([1.0, 2.0, 4.0]) == pytest.approx(3 / (1 + 0.5 + 0.25))
    assert bench.harmonic([]) == 0.0
    assert bench.harmonic([0.0, 2.0]) == pytest.approx(2.0)   # failed roots drop out
    assert bench.pct([1.0, 2.0, 3.0, 4.0, 5.0], 50) == 3.0


def test_host_cpu_reports_model_and_threads():
    model, nproc = bench.host_cpu()
    assert isinstance(model, str) and model
    assert nproc >= 1


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""
