"""Pins for the SpMSpV oracle (CPU only).

* The worked example of the paper's node-local matrix figure (section 4.1):
  DCSC arrays derived by hand from the printed nonzero pattern, and
  hand-computed (select, min) products.
* Dense brute force on small random blocks.
* BFS driven by repeated products plus the complement mask and parent
  update of Algorithm 3 reproduces the queue BFS, on the whole matrix and on
  an emulated p_r x p_c processor grid.
"""
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig3_dcsc.json")


def load_fig3():
    with open(GOLDEN) as f:
        return json.load(f)


def fig3_dense():
    fx = load_fig3()
    a = np.zeros((6, 6), dtype=bool)
    for r, cols in fx["pattern_rows"].items():
        a[int(r), cols] = True
    return a


def test_fig3_dcsc_arrays():
    fx = load_fig3()
    a = fig3_dense()
    whole = graphgen.dcsc_from_dense(a)
    assert whole.jc.tolist() == fx["whole"]["jc"]
    assert whole.cp.tolist() == fx["whole"]["cp"]
    assert whole.ir.tolist() == fx["whole"]["ir"]
    t0 = graphgen.dcsc_from_dense(a[0:3])
    assert (t0.jc.tolist(), t0.cp.tolist(), t0.ir.tolist()) == (
        fx["thread0_rows_0_2"]["jc"], fx["thread0_rows_0_2"]["cp"], fx["thread0_rows_0_2"]["ir"])
    t1 = graphgen.dcsc_from_dense(a[3:6])
    assert (t1.jc.tolist(), t1.cp.tolist(), t1.ir.tolist()) == (
        fx["thread1_rows_3_5_local"]["jc"], fx["thread1_rows_3_5_local"]["cp"],
        fx["thread1_rows_3_5_local"]["ir"])


def test_fig3_products():
    fx = load_fig3()
    w = fx["whole"]
    for case in fx["products"]:
        idx, val = oracle.spmspv(6, 6, w["jc"], w["cp"], w["ir"], case["frontier"])
        assert idx.tolist() == case["out_idx"]
        assert val.tolist() == case["out_val"]


def test_fig3_row_split_matches_whole():
    """The two thread pieces of the figure give the whole product when their
    local row ids are shifted back (rows 3-5 are local rows 0-2)."""
    fx = load_fig3()
    t0, t1 = fx["thread0_rows_0_2"], fx["thread1_rows_3_5_local"]
    for case in fx["products"]:
        i0, v0 = oracle.spmspv(3, 6, t0["jc"], t0["cp"], t0["ir"], case["frontier"])
        i1, v1 = oracle.spmspv(3, 6, t1["jc"], t1["cp"], t1["ir"], case["frontier"])
        assert np.concatenate([i0, i1 + 3]).tolist() == case["out_idx"]
        assert np.concatenate([v0, v1]).tolist() == case["out_val"]


def dense_spmspv(a, fidx, fval):
    """out[r] = min over k in f with a[r, k] of val(k); dense brute force."""
    big = np.iinfo(np.int64).max
    vals = np.full(a.shape[1], big, dtype=np.int64)
    vals[np.asarray(fidx, dtype=np.int64)] = np.asarray(fval, dtype=np.int64)
    m = np.where(a, vals[None, :], big).min(axis=1)
    idx = np.nonzero(m != big)[0]
    return idx.astype(np.int32), m[idx].astype(np.int32)


@pytest.mark.parametrize("seed", range(12))
def test_dense_brute_force(seed):
    rng = np.random.default_rng(seed)
    nr = int(rng.integers(1, 257))
    nc = int(rng.integers(1, 257))
    dens = float(rng.choice([0.002, 0.01, 0.05, 0.2]))
    a = rng.random((nr, nc)) < dens
    blk = graphgen.dcsc_from_dense(a)
    k = int(rng.integers(0, nc + 1))
    fidx = np.sort(rng.choice(nc, size=k, replace=False)).astype(np.int32)
    use_vals = seed % 2 == 1
    fval = rng.integers(0, 1 << 30, size=k).astype(np.int32) if use_vals else fidx
    idx, val = oracle.spmspv(nr, nc, blk.jc, blk.cp, blk.ir, fidx, fval if use_vals else None)
    bi, bv = dense_spmspv(a, fidx, fval)
    assert np.array_equal(idx, bi)
    assert np.array_equal(val, bv)


def test_empty_and_empty_columns():
    a = np.zeros((5, 5), dtype=bool)
    a[1, 2] = a[3, 2] = a[0, 4] = True
    blk = graphgen.dcsc_from_dense(a)
    assert blk.jc.tolist() == [2, 4]
    idx, val = oracle.spmspv(5, 5, blk.jc, blk.cp, blk.ir, [])
    assert idx.size == 0 and val.size == 0
    idx, val = oracle.spmspv(5, 5, blk.jc, blk.cp, blk.ir, [0, 1, 3])
    assert idx.size == 0
    idx, val = oracle.spmspv(5, 5, blk.jc, blk.cp, blk.ir, [0, 2, 4])
    assert idx.tolist() == [0, 1, 3] and val.tolist() == [4, 2, 2]


def test_generated_block_sampled_rows():
    """A generated hypersparse block: sampled rows checked one by one."""
    blk = graphgen.dcsc_block(16, 20000, 9)
    f = graphgen.frontier_sample(16, 6554, 4)
    idx, val = oracle.spmspv_block(blk, f)
    assert np.all(np.diff(idx) > 0)
    fset = set(f.tolist())
    cols_of_row = {}
    for p, c in enumerate(blk.jc):
        for q in range(blk.cp[p], blk.cp[p + 1]):
            cols_of_row.setdefault(int(blk.ir[q]), []).append(int(c))
    expect = {}
    for r, cols in cols_of_row.items():
        hit = [c for c in cols if c in fset]
        if hit:
            expect[r] = min(hit)
    assert idx.tolist() == sorted(expect)
    assert val.tolist() == [expect[r] for r in sorted(expect)]


# ---------------------------------------------------------------- BFS through products
def csr_to_dcsc(g, r0=0, r1=None, c0=0, c1=None):
    """DCSC of the sub-block A[r0:r1, c0:c1] of a symmetric CSR adjacency
    (A(v, u) != 0 for every edge u -> v; local ids)."""
    r1 = g.n if r1 is None else r1
    c1 = g.n if c1 is None else c1
    jc, cp, ir = [], [0], []
    for u in range(c0, c1):
        nb = g.col[g.off[u]:g.off[u + 1]]
        rows = nb[(nb >= r0) & (nb < r1)] - r0
        if rows.size:
            jc.append(u - c0)
            ir.extend(rows.tolist())
            cp.append(len(ir))
    return graphgen.DCSCBlock(r1 - r0, c1 - c0, np.array(jc, np.int32),
                              np.array(cp, np.int32), np.array(ir, np.int32))


def bfs_2d_emulated(g, root, pr, pc):
    """Algorithm 3 on a host-emulated pr x pc grid. Collectives become array
    gathers: the frontier is gathered per processor column (expand), each
    block forms its local product, contributions are min-merged per row
    (fold), then the complement mask and parent update are applied."""
    n = g.n
    rb = [n * i // pr for i in range(pr + 1)]
    cb = [n * j // pc for j in range(pc + 1)]
    blocks = {(i, j): csr_to_dcsc(g, rb[i], rb[i + 1], cb[j], cb[j + 1])
              for i in range(pr) for j in range(pc)}
    parent = np.full(n, -1, np.int64)
    level = np.full(n, -1, np.int64)
    parent[root] = root
    level[root] = 0
    f = np.array([root], np.int64)
    k = 0
    while f.size:
        k += 1
        t = np.full(n, np.iinfo(np.int64).max, np.int64)
        for (i, j), blk in blocks.items():
            fj = f[(f >= cb[j]) & (f < cb[j + 1])] - cb[j]          # expand
            idx, val = oracle.spmspv_block(blk, fj.astype(np.int32))
            rows = idx.astype(np.int64) + rb[i]
            np.minimum.at(t, rows, val.astype(np.int64) + cb[j])    # fold
        hit = np.nonzero((t != np.iinfo(np.int64).max) & (parent == -1))[0]  # mask
        parent[hit] = t[hit]                                         # update
        level[hit] = k
        f = hit
    return parent.astype(np.int32), level.astype(np.int32)


@pytest.mark.parametrize("pr,pc", [(1, 1), (2, 2), (2, 3), (4, 4)])
def test_bfs_by_products_matches_queue_bfs(pr, pc):
    g = graphgen.rmat_csr(9, 8, 5)
    for root in graphgen.roots(g, 3, 55):
        p, lv = oracle.bfs_graph(g, int(root))
        p2, lv2 = bfs_2d_emulated(g, int(root), pr, pc)
        assert np.array_equal(lv, lv2)
        assert np.array_equal(p, p2)


def test_bfs_by_products_on_grid():
    g = graphgen.grid_csr(12)
    p, lv = oracle.bfs_graph(g, 40)
    p2, lv2 = bfs_2d_emulated(g, 40, 2, 3)
    assert np.array_equal(lv, lv2) and np.array_equal(p, p2)


def test_planted_max_semiring_is_caught():
    """A (select, max) product (the other reading of the semiring) differs
    from the golden min products: the fixture pins the choice of min."""
    fx = load_fig3()
    a = fig3_dense()
    case = fx["products"][0]
    f = np.array(case["frontier"])
    vals = np.where(a[:, f], f[None, :], -1).max(axis=1)
    got = [int(v) for v in vals if v >= 0]
    assert got != case["out_val"]


@pytest.mark.parametrize("pr,pc", [(1, 1), (2, 2), (2, 3), (4, 4), (3, 1), (1, 5)])
def test_bfs_2d_equals_queue_bfs(pr, pc):
    """Algorithm 3 over a p_r x p_c grid of shares (the oracle's SpMSpV per
    share, min-fold per row block, mask) gives the queue BFS's parents and
    levels: undirected R-MAT, a grid, and a directed graph."""
    rng = np.random.default_rng(pr * 10 + pc)
    graphs = [graphgen.rmat_csr(10, 8, 3 + pr), graphgen.grid_csr(17, 9)]
    n = 700
    src, dst = rng.integers(0, n, 4000), rng.integers(0, n, 4000)
    order = np.lexsort((dst, src))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(src[order], minlength=n))
    graphs.append(graphgen.CSR(n, off, dst[order].astype(np.int32)))
    for g in graphs:
        R, C, shares = graphgen.csr_to_2d(g, pr, pc)
        assert sum(s.nnz for s in shares) == g.nnz
        for r in graphgen.roots(g, 3, 7):
            p2, l2 = oracle.bfs_2d(g.n, R, C, pr, pc, shares, int(r))
            p1, l1 = oracle.bfs_graph(g, int(r))
            assert np.array_equal(p2, p1) and np.array_equal(l2, l1)
