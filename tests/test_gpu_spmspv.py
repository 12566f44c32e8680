"""GPU parity of bfs_spmspv (DCSC share) against the CPU oracle."""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import gpu_spmspv, say, torch_cuda
from paper_1104_4518_amd import bfs as B

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig3_dcsc.json")


def block_on_device(b, sort_max=0):
    Gb = B.Graph.from_dcsc(b.nrows, b.ncols, b.jc, b.cp, b.ir)
    if sort_max:
        Gb.set_options(spmspv_sort_max=sort_max)
    return Gb


# both branches of the polyalgorithm: -1 = the binned accumulator only,
# 8192 = the sort path for frontiers up to 8192 entries
PATHS = pytest.mark.parametrize("path", [-1, 8192], ids=["binned", "sort"])


def check(Gb, blk, fidx, fval=None):
    gi, gv = gpu_spmspv(Gb, fidx, fval)
    oi, ov = oracle.spmspv_block(blk, fidx, fval)
    assert np.array_equal(gi, oi)
    assert np.array_equal(gv, ov)
    return gi


def test_fig3_worked_example():
    with open(GOLDEN) as f:
        fx = json.load(f)
    w = fx["whole"]
    blk = graphgen.DCSCBlock(6, 6, np.array(w["jc"], np.int32), np.array(w["cp"], np.int32),
                             np.array(w["ir"], np.int32))
    Gb = block_on_device(blk)
    for case in fx["products"]:
        say(f"fig3 frontier {case['frontier']}")
        gi, gv = gpu_spmspv(Gb, np.array(case["frontier"], np.int32))
        assert gi.tolist() == case["out_idx"]
        assert gv.tolist() == case["out_val"]


@PATHS
@pytest.mark.parametrize("seed", range(6))
def test_random_small_blocks(seed, path):
    rng = np.random.default_rng(seed)
    nr, nc = int(rng.integers(1, 3000)), int(rng.integers(1, 3000))
    a = rng.random((nr, nc)) < float(rng.choice([0.0005, 0.003, 0.02]))
    blk = graphgen.dcsc_from_dense(a)
    Gb = block_on_device(blk, path)
    for rep in range(3):
        k = int(rng.integers(0, nc + 1))
        f = np.sort(rng.choice(nc, size=k, replace=False)).astype(np.int32)
        fv = rng.integers(-(1 << 30), 1 << 30, size=k).astype(np.int32) if rep == 2 else None
        say(f"random block seed {seed} rep {rep} k {k}")
        check(Gb, blk, f, fv)


@PATHS
def test_edge_cases_and_errors(path):
    a = np.zeros((70, 90), dtype=bool)
    a[3, 5] = a[60, 5] = a[7, 89] = a[0, 40] = True
    blk = graphgen.dcsc_from_dense(a)
    Gb = block_on_device(blk, path)
    say("empty frontier")
    assert check(Gb, blk, np.zeros(0, np.int32)).size == 0
    say("only empty columns")
    assert check(Gb, blk, np.array([0, 1, 88], np.int32)).size == 0
    say("max index")
    check(Gb, blk, np.array([5, 89], np.int32))
    # unsorted / duplicate / out-of-range frontier -> BFS_ERR_ARG
    for bad in ([5, 3], [5, 5], [90], [-1, 5]):
        say(f"bad frontier {bad}")
        with pytest.raises(B.BfsError) as ei:
            gpu_spmspv(Gb, np.array(bad, np.int32))
        assert ei.value.code == B.BFS_ERR_ARG
    # capacity too small -> BFS_ERR_CAPACITY with the size needed
    say("capacity")
    with pytest.raises(B.BfsError) as ei:
        gpu_spmspv(Gb, np.array([5, 40, 89], np.int32), capacity=2)
    assert ei.value.code == B.BFS_ERR_CAPACITY and "need 4" in str(ei.value)
    # the accumulator is clean after the failures
    check(Gb, blk, np.array([5, 40, 89], np.int32))
    check(Gb, blk, np.arange(90, dtype=np.int32))


@PATHS
def test_empty_block(path):
    blk = graphgen.DCSCBlock(10, 10, np.zeros(0, np.int32), np.zeros(1, np.int32),
                             np.zeros(0, np.int32))
    Gb = block_on_device(blk, path)
    assert check(Gb, blk, np.array([1, 2], np.int32)).size == 0


def test_bad_dcsc_rejected():
    jc = np.array([1, 1], np.int32)
    cp = np.array([0, 1, 2], np.int32)
    ir = np.array([0, 1], np.int32)
    with pytest.raises(B.BfsError) as ei:
        B.Graph.from_dcsc(4, 4, jc, cp, ir)
    assert ei.value.code == B.BFS_ERR_FORMAT
    with pytest.raises(B.BfsError) as ei:
        B.Graph.from_dcsc(4, 4, np.array([1, 2], np.int32), cp, np.array([0, 4], np.int32))
    assert ei.value.code == B.BFS_ERR_FORMAT


@PATHS
@pytest.mark.parametrize("density", [0.0001, 0.001, 0.01, 0.1])
def test_generated_block_scale20(density, path):
    blk = graphgen.dcsc_block(20, 1 << 18, 12)
    Gb = block_on_device(blk, path)
    k = int(density * (1 << 20))
    for s in range(2):
        f = graphgen.frontier_sample(20, k, 300 + s)
        say(f"block2^20 density {density} call {s}")
        check(Gb, blk, f)


def test_config_share_2pow26():
    """The benchmarked share: 2^26 x 2^26, 16.8M uniform nonzeros (256 row
    bins), ten calls at each of the four densities, element-wise against the
    oracle (the bins, their cursors and the chained scan are reused by every
    call). The share's own tuned switch decides the branch, as in the
    benchmark."""
    blk = graphgen.dcsc_block(26, 1 << 24, 4)
    Gb = block_on_device(blk)
    Gb.tune()
    call = 0
    for density in (0.0001, 0.001, 0.01, 0.1):
        k = int(density * (1 << 26))
        for rep in range(10):
            f = graphgen.frontier_sample(26, k, 4000 + call)
            call += 1
            say(f"share 2^26 density {density} call {rep}")
            out = check(Gb, blk, f)
            assert out.size > 0


def test_bins_over_the_lds_accumulator_use_the_block_spa():
    """One bin of 2^18 rows receiving more distinct rows than its LDS
    accumulator ranks (16384): those bins take the minimum through the
    block-wide accumulator and must leave it clean; neighbouring bins stay in
    LDS. Values repeat so many rows see several candidates."""
    rng = np.random.default_rng(21)
    nr, nc, nnz = 3 * (1 << 18) + 5, 1 << 17, 1 << 21
    rows = rng.integers(0, nr, nnz)
    # crowd the middle bin: most entries land in rows [2^18, 2^19)
    crowd = rng.random(nnz) < 0.7
    rows[crowd] = rng.integers(1 << 18, 1 << 19, int(crowd.sum()))
    cols = rng.integers(0, nc, nnz)
    key = np.unique(cols.astype(np.int64) << 32 | rows.astype(np.int64))
    c, r = (key >> 32).astype(np.int64), (key & 0xFFFFFFFF).astype(np.int32)
    jc, start = np.unique(c, return_index=True)
    blk = graphgen.DCSCBlock(nr, nc, jc.astype(np.int32),
                             np.append(start, r.size).astype(np.int32), r)
    Gb = block_on_device(blk, -1)
    for rep, k in enumerate((nc // 2, 3000, nc // 2, nc)):
        f = np.sort(rng.choice(nc, size=k, replace=False)).astype(np.int32)
        fv = rng.integers(-50, 50, size=k).astype(np.int32) if rep != 1 else None
        say(f"crowded bin rep {rep} k {k}")
        out = check(Gb, blk, f, fv)
        if rep == 0:
            mid = ((out >= (1 << 18)) & (out < (1 << 19))).sum()
            assert mid > 16384   # the LDS accumulator's limit is exceeded


def test_many_bins_and_products_in_one_bin():
    """64 row bins, a frontier whose products all fall into one late bin (the
    chained scan must carry the empty bins before it), then products spread
    over every bin; and repeated calls that alternate between them."""
    rng = np.random.default_rng(5)
    nr, nc = 64 * (1 << 18), 5000
    rows_a = rng.integers(60 * (1 << 18), 61 * (1 << 18), 20000)   # one bin
    rows_b = rng.integers(0, nr, 20000)
    cols = np.concatenate([rng.integers(0, nc // 2, 20000), rng.integers(nc // 2, nc, 20000)])
    rows = np.concatenate([rows_a, rows_b])
    key = np.unique(cols.astype(np.int64) << 32 | rows.astype(np.int64))
    c, r = (key >> 32).astype(np.int64), (key & 0xFFFFFFFF).astype(np.int32)
    jc, start = np.unique(c, return_index=True)
    blk = graphgen.DCSCBlock(nr, nc, jc.astype(np.int32),
                             np.append(start, r.size).astype(np.int32), r)
    Gb = block_on_device(blk, -1)
    first = np.arange(0, nc // 2, dtype=np.int32)
    second = np.arange(nc // 2, nc, dtype=np.int32)
    for rep in range(3):
        say(f"one late bin rep {rep}")
        out = check(Gb, blk, first)
        assert out.size > 0 and out.min() >= 60 * (1 << 18) and out.max() < 61 * (1 << 18)
        say(f"all bins rep {rep}")
        check(Gb, blk, second)
        check(Gb, blk, np.arange(nc, dtype=np.int32))


def test_sort_path_limits_and_fallback():
    """Frontiers of 8192 entries (the sort path's limit) and 8193 (the
    accumulator), a product above 8192 pairs from a small frontier (the sort
    path hands over to the accumulator), min over many candidates per row, and
    calls alternating between the two paths on one handle."""
    rng = np.random.default_rng(9)
    a = rng.random((400, 20000)) < 0.002
    blk = graphgen.dcsc_from_dense(a)
    Gb = block_on_device(blk)
    for k in (8192, 8193, 1, 0):
        f = np.sort(rng.choice(20000, size=k, replace=False)).astype(np.int32)
        say(f"sort limit frontier {k}")
        check(Gb, blk, f)
    dense = np.zeros((3000, 64), dtype=bool)
    dense[:, :] = rng.random((3000, 64)) < 0.9   # ~172K products from 64 columns
    bd = graphgen.dcsc_from_dense(dense)
    Gd = block_on_device(bd)
    for rep in range(3):
        f = np.sort(rng.choice(64, size=int(rng.integers(8, 64)), replace=False)).astype(np.int32)
        fv = rng.integers(-1000, 1000, size=f.size).astype(np.int32)
        say(f"fallback product rep {rep}")
        check(Gd, bd, f, fv)
        check(Gd, bd, f[:2])


def test_buckets_without_a_record_fall_back_to_the_column_search():
    """Scattered lookups read a record per bucket of columns; a bucket with
    more stored columns than a record holds, or with a column longer than its
    16-bit row counts, has none and is searched in AUX, JC and CP, in the same
    waves as entries whose buckets have records. Here the buckets span 64
    columns: bucket 0 stores all 64, bucket 1 holds a column of 70,000 rows,
    the rest are sparse; small frontiers mix all three kinds."""
    rng = np.random.default_rng(71)
    nr, nc = 1 << 17, 1 << 16
    cols = set(range(64)) | {100}
    cols |= set(rng.choice(np.arange(128, nc), 2000, replace=False).tolist())
    jc = np.array(sorted(cols), np.int32)
    rows = []
    for c in jc:
        k = 70000 if c == 100 else int(rng.integers(1, 8))
        rows.append(np.sort(rng.choice(nr, k, replace=False)).astype(np.int32))
    cp = np.zeros(len(jc) + 1, np.int32)
    cp[1:] = np.cumsum([len(r) for r in rows])
    blk = graphgen.DCSCBlock(nr, nc, jc, cp, np.concatenate(rows))
    Gb = block_on_device(blk, -1)
    stored = jc.astype(np.int64)
    for seed in range(4):
        r2 = np.random.default_rng(100 + seed)
        pick = set(r2.choice(64, 10, replace=False).tolist()) | {100}
        pick |= set(r2.choice(stored, 300, replace=False).tolist())
        pick |= set(r2.choice(nc, 100, replace=False).tolist())   # some on empty columns
        fidx = np.array(sorted(pick), np.int32)
        fval = r2.integers(-(1 << 30), 1 << 30, len(fidx)).astype(np.int32) if seed % 2 else None
        say(f"record fallback frontier {len(fidx)} seed {seed}")
        check(Gb, blk, fidx, fval)
    check(Gb, blk, jc.copy())   # every stored column
