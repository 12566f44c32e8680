"""bfs_tune: the choices it makes, its cache file, and unchanged results."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import assert_bfs_equal, gpu_spmspv, say
from paper_1104_4518_amd import bfs as B

pytestmark = pytest.mark.gpu


def test_tune_csr_choices_cache_and_results(tmp_path):
    g = graphgen.rmat_csr(14, 16, 41)
    cache = tmp_path / "tune.txt"
    G = B.Graph.from_csr(g.n, g.off, g.col)
    say("tune rmat14")
    G.tune(str(cache))
    o = G.get_options()
    assert o.batch_levels in (4, 8)
    ct_low = max(g.n // 512, 4096)
    assert (o.claim_min_frontier, o.claim_threshold) in (
        (4096, 0), (1024, 0), (16384, 0), (32, ct_low), (1024, ct_low), (4096, g.nnz // 16))
    assert o.pull_alpha in (4, 14, 40)
    assert o.grid_blocks > 0 and o.grid_blocks % 2 == 0
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and " csr n=16384 " in lines[0] and "min_frontier=" in lines[0]
    assert "pull_alpha=" in lines[0] and "claim_threshold=" in lines[0]
    assert o.small_frontier in (8192, 1024, -1) and "small_frontier=" in lines[0]
    for r in graphgen.roots(g, 3, 5):
        say(f"tuned rmat14 root {r}")
        assert_bfs_equal(g, G, r)
    # a second handle of the same shape takes the cached choice
    G2 = B.Graph.from_csr(g.n, g.off, g.col)
    G2.tune(str(cache))
    o2 = G2.get_options()
    assert (o2.grid_blocks, o2.batch_levels, o2.claim_min_frontier, o2.pull_alpha,
            o2.claim_threshold, o2.small_frontier) == \
        (o.grid_blocks, o.batch_levels, o.claim_min_frontier, o.pull_alpha, o.claim_threshold,
         o.small_frontier)
    assert len(cache.read_text().splitlines()) == 1


def test_tune_dcsc_polyalgorithm_switch(tmp_path):
    blk = graphgen.dcsc_block(20, 1 << 18, 12)
    Gb = B.Graph.from_dcsc(blk.nrows, blk.ncols, blk.jc, blk.cp, blk.ir)
    cache = tmp_path / "tune.txt"
    say("tune dcsc 2^20")
    Gb.tune(str(cache))
    assert Gb.get_options().spmspv_sort_max in (-1, 64, 512, 2048, 8192)
    line = cache.read_text().splitlines()[0]
    assert " dcsc 1048576x1048576 " in line and "sort_max=" in line
    for k in (10, 3000, 20000):
        f = graphgen.frontier_sample(20, k, 900 + k)
        say(f"tuned dcsc frontier {k}")
        gi, gv = gpu_spmspv(Gb, f)
        oi, ov = oracle.spmspv_block(blk, f)
        assert np.array_equal(gi, oi) and np.array_equal(gv, ov)


def test_tune_csr_repeats_its_choice():
    """Three tunings of one graph (no cache) pick the same options: a value
    replaces the current one only when it is clearly faster."""
    g = graphgen.rmat_csr(18, 16, 44)
    G = B.Graph.from_csr(g.n, g.off, g.col)
    picks = []
    for i in range(3):
        say(f"tune rmat18 pass {i}")
        G.tune()
        o = G.get_options()
        picks.append((o.grid_blocks, o.batch_levels, o.claim_min_frontier, o.pull_alpha,
                      o.claim_threshold, o.small_frontier))
    assert picks[0] == picks[1] == picks[2], picks
