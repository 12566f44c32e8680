"""Pins for the BFS oracle (CPU only).

The oracle is checked against things other than itself: brute-force
all-pairs distances, closed forms of textbook graphs, a library routine
(scipy's shortest paths), union-find component sizes, and the minimum-id
parent definition evaluated directly from the levels. Each pin is chosen so
that a plausible slip in the oracle (a dropped min update, an off-by-one
level, a wrong queue order) fails at least one of them.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import graphgen
import oracle


# ---------------------------------------------------------------- helpers
def brute_force(n, edges, root):
    """Levels by Floyd-Warshall on a dense matrix and parents by definition."""
    inf = np.iinfo(np.int64).max // 4
    d = np.full((n, n), inf, dtype=np.int64)
    np.fill_diagonal(d, 0)
    adj = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            d[u, v] = d[v, u] = 1
            adj[u].add(v)
            adj[v].add(u)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    level = np.where(d[root] >= inf, -1, d[root]).astype(np.int32)
    parent = np.full(n, -1, np.int32)
    parent[root] = root
    for v in range(n):
        if level[v] > 0:
            parent[v] = min(u for u in adj[v] if level[u] == level[v] - 1)
    return parent, level


def min_parent_from_levels(g, level, root):
    """parent[v] = min{u in N(v) : level[u] = level[v] - 1}, vectorised."""
    n = g.n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.off))
    dst = g.col.astype(np.int64)
    ok = (level[src] >= 1) & (level[dst] == level[src] - 1)
    parent = np.full(n, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(parent, src[ok], dst[ok])
    parent[parent == np.iinfo(np.int64).max] = -1
    parent[root] = root
    return parent.astype(np.int32)


def union_find_sizes(n, edges):
    p = list(range(n))

    def find(x):
        while p[x] != x:
            p[x] = p[p[x]]
            x = p[x]
        return x

    for u, v in edges:
        ru, rv = find(u), find(v)
        if ru != rv:
            p[ru] = rv
    roots = [find(x) for x in range(n)]
    return {x: roots.count(roots[x]) for x in range(n)}


def run(g, root):
    return oracle.bfs(g.n, g.off, g.col, root)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_small_graphs(n):
    """Every labelled graph on n <= 5 vertices, every root."""
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        g = graphgen.from_edges(n, edges)
        for root in range(n):
            p, lv = run(g, root)
            bp, bl = brute_force(n, edges, root)
            assert np.array_equal(lv, bl), (n, edges, root)
            assert np.array_equal(p, bp), (n, edges, root)


def test_random_graphs_up_to_64():
    rng = np.random.default_rng(7)
    for t in range(150):
        n = int(rng.integers(1, 65))
        m = int(rng.integers(0, 3 * n + 1))
        edges = [tuple(map(int, rng.integers(0, n, 2))) for _ in range(m)]
        g = graphgen.from_edges(n, edges)
        root = int(rng.integers(0, n))
        p, lv = run(g, root)
        bp, bl = brute_force(n, edges, root)
        assert np.array_equal(lv, bl), t
        assert np.array_equal(p, bp), t


# ---------------------------------------------------------------- closed forms
def test_path_from_end():
    n = 50
    g = graphgen.from_edges(n, [(i, i + 1) for i in range(n - 1)])
    p, lv = run(g, 0)
    assert lv.tolist() == list(range(n))
    assert p.tolist() == [0] + list(range(n - 1))


def test_path_from_middle():
    n = 11
    g = graphgen.from_edges(n, [(i, i + 1) for i in range(n - 1)])
    p, lv = run(g, 5)
    assert lv.tolist() == [abs(i - 5) for i in range(n)]
    assert p.tolist() == [i + 1 if i < 5 else (5 if i == 5 else i - 1) for i in range(n)]


@pytest.mark.parametrize("n", [3, 4, 7, 10])
def test_cycle(n):
    g = graphgen.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
    p, lv = run(g, 0)
    assert lv.tolist() == [min(i, n - i) for i in range(n)]
    exp = [0]
    for i in range(1, n):
        cands = [u for u in ((i - 1) % n, (i + 1) % n) if min(u, n - u) == min(i, n - i) - 1]
        exp.append(min(cands))
    assert p.tolist() == exp


def test_star():
    n = 9
    g = graphgen.from_edges(n, [(0, i) for i in range(1, n)])
    p, lv = run(g, 0)
    assert lv.tolist() == [0] + [1] * (n - 1)
    assert p.tolist() == [0] * n
    p, lv = run(g, 4)
    assert lv.tolist() == [1] + [2] * 3 + [0] + [2] * 4
    assert p.tolist() == [4, 0, 0, 0, 4, 0, 0, 0, 0]


def test_complete_graph():
    n = 12
    g = graphgen.from_edges(n, itertools.combinations(range(n), 2))
    for r in (0, 5, 11):
        p, lv = run(g, r)
        assert lv.tolist() == [0 if i == r else 1 for i in range(n)]
        assert p.tolist() == [r] * n


def test_binary_tree():
    n = 127
    g = graphgen.from_edges(n, [(i, (i - 1) // 2) for i in range(1, n)])
    p, lv = run(g, 0)
    assert lv.tolist() == [int(np.floor(np.log2(i + 1))) for i in range(n)]
    assert p.tolist() == [0] + [(i - 1) // 2 for i in range(1, n)]


@pytest.mark.parametrize("w,r,c", [(8, 0, 0), (8, 3, 5), (17, 16, 2), (1, 0, 0)])
def test_grid_closed_form(w, r, c):
    g = graphgen.grid_csr(w)
    root = r * w + c
    p, lv = run(g, root)
    ids = np.arange(w * w)
    i, j = ids // w, ids % w
    assert np.array_equal(lv, np.abs(i - r) + np.abs(j - c))
    exp = np.where(i > r, ids - w, np.where(j > c, ids - 1, np.where(j < c, ids + 1,
                                                                     np.where(i < r, ids + w, ids))))
    assert np.array_equal(p, exp)


def test_disconnected_and_isolated_root():
    g = graphgen.from_edges(6, [(0, 1), (1, 2), (3, 4)])
    p, lv = run(g, 5)
    assert lv.tolist() == [-1] * 5 + [0]
    assert p.tolist() == [-1] * 5 + [5]
    p, lv = run(g, 3)
    assert lv.tolist() == [-1, -1, -1, 0, 1, -1]
    assert p.tolist() == [-1, -1, -1, 3, 3, -1]


def test_bad_root_rejected():
    g = graphgen.from_edges(3, [(0, 1)])
    with pytest.raises(ValueError):
        oracle.bfs(g.n, g.off, g.col, 3)
    with pytest.raises(ValueError):
        oracle.bfs(g.n, g.off, g.col, -1)


# ---------------------------------------------------------------- library / invariants
def test_component_sizes_union_find():
    rng = np.random.default_rng(11)
    n = 300
    edges = [tuple(map(int, rng.integers(0, n, 2))) for _ in range(220)]
    g = graphgen.from_edges(n, edges)
    sizes = union_find_sizes(n, edges)
    for root in rng.integers(0, n, 25):
        _, lv = run(g, int(root))
        assert int((lv >= 0).sum()) == sizes[int(root)]


def _scipy_levels(g, root):
    a = sp.csr_matrix((np.ones(g.nnz), g.col, g.off), shape=(g.n, g.n))
    d = shortest_path(a, unweighted=True, indices=[root])[0]
    return np.where(np.isinf(d), -1, d).astype(np.int32)


@pytest.mark.parametrize("scale,seed", [(8, 3), (10, 4), (12, 1)])
def test_rmat_against_scipy_and_definition(scale, seed):
    g = graphgen.rmat_csr(scale, 16, seed)
    for root in graphgen.roots(g, 6, 1000 + seed):
        p, lv = run(g, int(root))
        assert np.array_equal(lv, _scipy_levels(g, int(root)))
        assert np.array_equal(p, min_parent_from_levels(g, lv, int(root)))
        assert oracle.check_bfs(g, int(root), p, lv) == (0, -1)


def test_rmat12_config_all_roots():
    """The R-MAT scale-12 configuration with its 16 seeded roots."""
    g = graphgen.config_graph("rmat12")
    roots = graphgen.config_roots("rmat12", g)
    assert len(roots) == 16
    ncomp, labels = connected_components(
        sp.csr_matrix((np.ones(g.nnz), g.col, g.off), shape=(g.n, g.n)), directed=False)
    for root in roots:
        p, lv = run(g, int(root))
        assert int((lv >= 0).sum()) == int((labels == labels[root]).sum())
        assert np.array_equal(lv, _scipy_levels(g, int(root)))
        assert np.array_equal(p, min_parent_from_levels(g, lv, int(root)))
        # every tree edge exists in the graph
        reached = np.nonzero((lv > 0))[0]
        for v in reached[:200]:
            assert p[v] in g.col[g.off[v]:g.off[v + 1]]


def test_grid_512_levels_and_parents():
    g = graphgen.grid_csr(512)
    root = 512 * 100 + 300
    p, lv = run(g, root)
    ids = np.arange(g.n)
    i, j = ids // 512, ids % 512
    assert np.array_equal(lv, np.abs(i - 100) + np.abs(j - 300))
    assert lv.max() == (511 - 100) + 300
    assert oracle.check_bfs(g, root, p, lv) == (0, -1)


def test_reached_edges_counts_component_edges():
    g = graphgen.from_edges(7, [(0, 1), (1, 2), (2, 0), (3, 4), (5, 6)])
    _, lv = run(g, 0)
    assert oracle.reached_edges(g, lv) == 3
    _, lv = run(g, 5)
    assert oracle.reached_edges(g, lv) == 1


# ---------------------------------------------------------------- planted mistakes
def _first_visit_bfs(g, root):
    """A BFS that keeps the first-found parent: what the oracle would be with
    its min update dropped."""
    n = g.n
    lv = np.full(n, -1, np.int32)
    p = np.full(n, -1, np.int32)
    lv[root] = 0
    p[root] = root
    q = [root]
    h = 0
    while h < len(q):
        u = q[h]
        h += 1
        for v in g.col[g.off[u]:g.off[u + 1]][::-1]:   # reverse scan order
            if lv[v] == -1:
                lv[v] = lv[u] + 1
                p[v] = u
                q.append(int(v))
    return p, lv


def test_pins_catch_dropped_min_update():
    g = graphgen.rmat_csr(10, 16, 4)
    root = int(graphgen.roots(g, 1, 99)[0])
    p_bad, lv = _first_visit_bfs(g, root)
    assert not np.array_equal(p_bad, min_parent_from_levels(g, lv, root))
    assert oracle.check_bfs(g, root, p_bad, lv)[0] == 6


def test_checker_catches_planted_level_and_parent_errors():
    g = graphgen.rmat_csr(10, 16, 4)
    root = int(graphgen.roots(g, 1, 99)[0])
    p, lv = run(g, root)
    assert oracle.check_bfs(g, root, p, lv) == (0, -1)
    reached = np.nonzero(lv > 1)[0]
    v = int(reached[0])
    lv2 = lv.copy()
    lv2[v] += 1
    assert oracle.check_bfs(g, root, p, lv2)[0] in (4, 5, 6)
    p2 = p.copy()
    p2[v] = root
    assert oracle.check_bfs(g, root, p2, lv)[0] == 6
    unreached = np.nonzero(lv == -1)[0]
    if unreached.size:
        lv3, p3 = lv.copy(), p.copy()
        u = int(unreached[0])
        lv3[u], p3[u] = 1, root
        assert oracle.check_bfs(g, root, p3, lv3)[0] != 0
    lv4, p4 = lv.copy(), p.copy()
    lv4[v], p4[v] = -1, -1
    assert oracle.check_bfs(g, root, p4, lv4)[0] == 3
