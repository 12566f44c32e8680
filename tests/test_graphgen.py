"""Seeded input generators: determinism and the shape of the workloads."""
import numpy as np

import graphgen


def test_rmat_deterministic_and_seeded():
    a = graphgen.rmat_csr(12, 16, 1)
    b = graphgen.rmat_csr(12, 16, 1)
    c = graphgen.rmat_csr(12, 16, 2)
    assert a.hash() == b.hash()
    assert a.hash() != c.hash()


def test_csr_well_formed():
    g = graphgen.rmat_csr(12, 16, 1)
    assert g.off[0] == 0 and g.off[-1] == g.nnz
    assert np.all(np.diff(g.off) >= 0)
    assert g.col.min() >= 0 and g.col.max() < g.n
    for v in range(0, g.n, 37):
        row = g.col[g.off[v]:g.off[v + 1]]
        assert np.all(np.diff(row) > 0)        # sorted, no duplicates
        assert v not in row                     # no self-loops
    # symmetric: (u, v) present iff (v, u) present
    src = np.repeat(np.arange(g.n), np.diff(g.off))
    fwd = set(zip(src.tolist(), g.col.tolist()))
    assert all((v, u) in fwd for (u, v) in list(fwd)[:5000])


def test_rmat_shape_statistics():
    """Unique-edge and isolated-vertex fractions of a Graph 500-style R-MAT."""
    g = graphgen.rmat_csr(16, 16, 1)
    uniq = g.nnz / 2 / (16 << 16)
    iso = float((g.degrees() == 0).mean())
    assert 0.83 < uniq < 0.90
    assert 0.24 < iso < 0.34
    assert g.degrees().max() > 50 * g.degrees().mean()       # skewed


def test_er_shape_statistics():
    g = graphgen.er_csr(14, 16, 3)
    d = g.degrees()
    assert abs(d.mean() - 32) < 1.0
    assert (d == 0).mean() < 1e-3
    assert d.max() < 70


def test_edge_list_endpoints_in_range():
    us, vs = graphgen.edge_list(0, 10, 5000, 4)
    assert us.min() >= 0 and us.max() < 1024 and vs.max() < 1024
    us2, _ = graphgen.edge_list(0, 10, 5000, 4)
    assert np.array_equal(us, us2)


def test_permutation_is_bijection():
    for bits in (1, 2, 5, 10, 13):
        img = [graphgen.perm(x, bits, 7) for x in range(1 << bits)]
        assert sorted(img) == list(range(1 << bits))


def test_roots_distinct_degree_positive():
    g = graphgen.rmat_csr(12, 16, 1)
    r = graphgen.roots(g, 16, 1000)
    assert len(set(r.tolist())) == 16
    assert np.all(g.degrees()[r] >= 1)
    assert np.array_equal(r, graphgen.roots(g, 16, 1000))


def test_roots_when_few_candidates():
    g = graphgen.from_edges(10, [(0, 1)])
    r = graphgen.roots(g, 5, 3)
    assert sorted(r.tolist()) == [0, 1]


def test_grid_structure():
    g = graphgen.grid_csr(5, 3)
    assert g.n == 15 and g.nnz == 2 * (4 * 3 + 2 * 5)
    assert g.col[g.off[7]:g.off[8]].tolist() == [2, 6, 8, 12]
    assert g.col[g.off[0]:g.off[1]].tolist() == [1, 5]


def test_dcsc_block_well_formed():
    b = graphgen.dcsc_block(18, 50000, 6)
    assert b.nnz <= 50000 and b.nnz > 49000
    assert np.all(np.diff(b.jc) > 0)
    assert b.cp[0] == 0 and b.cp[-1] == b.nnz and np.all(np.diff(b.cp) > 0)
    for p in range(0, b.nzc, 97):
        seg = b.ir[b.cp[p]:b.cp[p + 1]]
        assert np.all(np.diff(seg) > 0)
    assert b.ir.min() >= 0 and b.ir.max() < b.nrows


def test_frontier_sample():
    f = graphgen.frontier_sample(20, 1000, 3)
    assert f.size == 1000 and np.all(np.diff(f) > 0) and f.max() < (1 << 20)
    assert np.array_equal(f, graphgen.frontier_sample(20, 1000, 3))
    assert graphgen.frontier_sample(20, 0, 3).size == 0


def test_upper_csr_stores_each_edge_once_and_closes_to_the_graph():
    g = graphgen.rmat_csr(10, 16, 3)
    u = graphgen.upper_csr(g)
    assert u.nnz * 2 == g.nnz   # symmetric, no self-loops: every edge in two rows
    src = np.repeat(np.arange(u.n), np.diff(u.off))
    assert (u.col > src).all()
    for r in range(u.n):   # rows ascending
        row = u.col[u.off[r]:u.off[r + 1]]
        assert (np.diff(row) > 0).all()
    # the symmetric closure of the stored half is the graph
    a = set(zip(src.tolist(), u.col.tolist()))
    closure = a | {(v, w) for (w, v) in a}
    gsrc = np.repeat(np.arange(g.n), np.diff(g.off))
    assert closure == set(zip(gsrc.tolist(), g.col.tolist()))
