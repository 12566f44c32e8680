"""The row-order evaluation of a level's masked product (every unvisited
vertex takes the first frontier vertex of its ascending row) reaches exactly
the queue BFS's parents and levels: closed forms, brute-force-sized random
graphs with many equal-level ties, R-MAT. CPU only."""
import numpy as np
import pytest

import graphgen
import oracle


def same(g, roots):
    for r in roots:
        p1, l1 = oracle.bfs_graph(g, int(r))
        p2, l2 = oracle.bfs_by_rows(g.n, g.off, g.col, int(r))
        assert np.array_equal(l1, l2), r
        assert np.array_equal(p1, p2), r


@pytest.mark.parametrize("name,edges,n", [
    ("path", [(i, i + 1) for i in range(30)], 31),
    ("cycle", [(i, (i + 1) % 17) for i in range(17)], 17),
    ("star", [(0, i) for i in range(1, 40)], 40),
    ("complete", [(i, j) for i in range(12) for j in range(i + 1, 12)], 12),
    ("two_components", [(0, 1), (1, 2), (3, 4), (4, 5), (5, 3)], 8),
])
def test_closed_form_graphs_every_root(name, edges, n):
    g = graphgen.from_edges(n, edges)
    same(g, range(n))


def test_grid_every_root():
    g = graphgen.grid_csr(9)
    same(g, range(g.n))


def test_random_graphs_with_ties():
    # dense small graphs: most vertices have several neighbours one level
    # up, so the min-id choice is exercised on every level
    rng = np.random.default_rng(11)
    for trial in range(60):
        n = int(rng.integers(2, 40))
        m = int(rng.integers(0, 4 * n))
        edges = list(zip(rng.integers(0, n, m).tolist(), rng.integers(0, n, m).tolist()))
        g = graphgen.from_edges(n, edges)
        same(g, rng.choice(n, min(n, 5), replace=False))


def test_rmat_scale_10():
    g = graphgen.rmat_csr(10, 16, 12)
    same(g, graphgen.roots(g, 6, 13))


def _rows_planted(n, off, col, root, immediate=False, last=False):
    """bfs_by_rows with a planted mistake: the level assigned during the
    scan (vertices found earlier in the level act as frontier), or the last
    frontier neighbour taken instead of the first."""
    parent = np.full(n, -1, np.int64)
    level = np.full(n, -1, np.int64)
    parent[root], level[root] = root, 0
    k, found = 0, True
    while found:
        k += 1
        found = []
        for v in range(n):
            if level[v] != -1:
                continue
            hits = [u for u in col[off[v]:off[v + 1]] if level[u] == k - 1]
            if hits:
                parent[v] = hits[-1] if last else hits[0]
                found.append(v)
                if immediate:
                    level[v] = k - 1   # wrongly visible to the rest of the scan
        for v in found:
            level[v] = k
    return parent.astype(np.int32), level.astype(np.int32)


@pytest.mark.parametrize("mistake", ["immediate", "last"])
def test_planted_mistakes_are_caught(mistake):
    g = graphgen.rmat_csr(10, 16, 12)
    caught = False
    for r in graphgen.roots(g, 6, 13):
        p1, l1 = oracle.bfs_graph(g, int(r))
        p2, l2 = _rows_planted(g.n, g.off, g.col, int(r), immediate=mistake == "immediate",
                               last=mistake == "last")
        caught |= not (np.array_equal(p1, p2) and np.array_equal(l1, l2))
    assert caught
