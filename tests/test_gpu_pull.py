"""GPU parity of the pull levels (the masked product computed by rows: every
unvisited vertex takes the first vertex one level up in its ascending
adjacency list) against the CPU oracle, bit for bit."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import assert_bfs_equal, gpu_bfs, graph_on_device, say, torch_cuda
from paper_1104_4518_amd import bfs as B

pytestmark = pytest.mark.gpu

# every level with a non-empty frontier pulls
ALWAYS = dict(claim=2, pull_alpha=1 << 30)


def pulled(G, g, roots, **opts):
    G.set_options(**{**ALWAYS, **opts})
    for r in roots:
        say(f"pull every level, root {r}, n={g.n}")
        _, ol = assert_bfs_equal(g, G, int(r))
        st = G.last_stats()
        assert st.pull_levels == st.levels, (st.pull_levels, st.levels)
        assert st.depth == ol.max()


@pytest.mark.parametrize("name,edges,n", [
    ("path", [(i, i + 1) for i in range(99)], 100),
    ("star", [(0, i) for i in range(1, 300)], 300),
    ("complete", [(i, j) for i in range(40) for j in range(i + 1, 40)], 40),
    ("two_components", [(0, 1), (1, 2), (3, 4), (4, 5), (5, 3)], 8),
    ("isolated", [], 5),
])
def test_pull_every_level_small_graphs(name, edges, n):
    g = graphgen.from_edges(n, edges)
    G = graph_on_device(g)
    pulled(G, g, range(n))


def test_pull_every_level_grid_and_rmat12():
    g = graphgen.grid_csr(33)
    pulled(graph_on_device(g), g, (0, 33 * 16 + 5, 33 * 33 - 1))
    g = graphgen.config_graph("rmat12")
    pulled(graph_on_device(g), g, graphgen.config_roots("rmat12", g))


@pytest.mark.parametrize("scale,seed", [(14, 31), (16, 32)])
def test_pull_every_level_rmat(scale, seed):
    g = graphgen.rmat_csr(scale, 16, seed)
    rng = np.random.default_rng(seed)
    roots = rng.choice(np.nonzero(np.diff(g.off) > 0)[0], 6, replace=False)
    pulled(graph_on_device(g), g, roots)


def test_pull_every_level_degree_ordered_copy():
    # n >= 2^20: the level kernels read the degree-ordered copy (pull scans
    # only its vertices of positive degree) and stage the hot prefix in LDS
    g = graphgen.rmat_csr(20, 16, 33)
    rng = np.random.default_rng(33)
    roots = rng.choice(np.nonzero(np.diff(g.off) > 0)[0], 3, replace=False)
    pulled(graph_on_device(g), g, roots)


def test_pull_every_level_graph_mode():
    g = graphgen.rmat_csr(14, 16, 34)
    rng = np.random.default_rng(34)
    roots = rng.choice(np.nonzero(np.diff(g.off) > 0)[0], 4, replace=False)
    pulled(graph_on_device(g), g, roots, mode=2)
    g = graphgen.grid_csr(64)
    pulled(graph_on_device(g), g, (0, 64 * 64 - 1), mode=2)


def test_default_policy_pulls_and_matches_push_only():
    """R-MAT's peak levels pull under the default policy; with the pull off
    (-1) and on, every root equals the oracle."""
    g = graphgen.rmat_csr(18, 16, 35)
    G = graph_on_device(g)
    rng = np.random.default_rng(35)
    roots = rng.choice(np.nonzero(np.diff(g.off) > 0)[0], 8, replace=False)
    pulls = 0
    for alpha in (-1, 14):
        G.set_options(pull_alpha=alpha)
        for r in roots:
            say(f"rmat18 pull_alpha {alpha} root {r}")
            assert_bfs_equal(g, G, int(r))
            st = G.last_stats()
            if alpha < 0:
                assert st.pull_levels == 0 and st.pull_edges == 0
            pulls += st.pull_levels
    assert pulls > 0


def test_er_pull():
    g = graphgen.er_csr(15, 16, 36)
    G = graph_on_device(g)
    rng = np.random.default_rng(36)
    roots = rng.choice(np.nonzero(np.diff(g.off) > 0)[0], 4, replace=False)
    for r in roots:
        say(f"er15 default root {r}")
        assert_bfs_equal(g, G, int(r))
    pulled(G, g, roots)


def test_pull_level_info_and_stats():
    torch = torch_cuda()
    g = graphgen.rmat_csr(16, 16, 37)
    G = graph_on_device(g)
    G.set_options(profile=1, claim=2, pull_alpha=1 << 30)
    r = int(np.argmax(np.diff(g.off)))
    say(f"rmat16 profiled pull root {r}")
    assert_bfs_equal(g, G, r)
    st = G.last_stats()
    info = [L for L in G.level_info() if L["frontier"] > 0]
    assert st.pull_levels == len(info) and all(L["mark"] == 2 for L in info)
    assert sum(L["pull_edges"] for L in info) == st.pull_edges
    # every level's searchers: the vertices of positive degree not yet reached
    p, lv = oracle.bfs_graph(g, r)
    deg = np.diff(g.off)
    for L in info:
        k = L["level"]
        unvisited = ((lv >= k) | (lv < 0)) & (deg > 0)
        assert L["pull_candidates"] == int(unvisited.sum()), k
        # each searcher reads at least one adjacency and at most its list
        assert L["pull_candidates"] <= L["pull_edges"] <= int(deg[unvisited].sum())
    assert st.pull_ms > 0.0
    G.set_options(pull_alpha=-1, claim=3, profile=-1)


def test_pull_alpha_validation():
    g = graphgen.from_edges(4, [(0, 1), (1, 2)])
    G = graph_on_device(g)
    with pytest.raises(B.BfsError):
        G.set_options(pull_alpha=-2)
    with pytest.raises(B.BfsError):
        G.set_options(pull_alpha=-2, cold_probe=2)
    # a rejected call applies none of its fields
    assert G.get_options().cold_probe == 3


@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_large_claim_levels_set_visited_bits_from_tags(kind):
    """With the mark levels disabled (edge floor 2^30) a symmetric graph's
    large frontiers are claimed; a claim level that reaches n/64 vertices or
    more sets the visited bits from its claimers' tags instead of one atomic
    per vertex. Every level after it must still see exactly the visited set."""
    g = graphgen.rmat_csr(16, 16, 38) if kind == "rmat" else graphgen.er_csr(16, 16, 38)
    G = graph_on_device(g)
    G.set_options(claim_threshold=1 << 30)
    rng = np.random.default_rng(38)
    roots = rng.choice(np.nonzero(np.diff(g.off) > 0)[0], 6, replace=False)
    for r in roots:
        say(f"{kind}16 claim levels only, root {r}")
        _, ol = assert_bfs_equal(g, G, int(r))
        st = G.last_stats()
        assert st.mark_levels == 0
        # some level reached at least n/64 vertices
        assert np.bincount(ol[ol >= 0]).max() * 64 >= g.n


def test_claim_level_with_many_new_vertices_from_few_edges():
    """A star of 2048 leaves beside a dense random part: from the centre,
    level 1 claims n/32 vertices through only 2048 adjacencies (well under
    nnz / 64, so not a touch-mark claim level) and sets their visited bits
    from the tags; the rest of the search must see exactly that set."""
    n = 1 << 16
    rng = np.random.default_rng(39)
    star = [(0, i) for i in range(1, 2049)]
    a = rng.integers(2049, n, 600000)
    b = rng.integers(2049, n, 600000)
    bridge = [(2048, 5000)]
    g = graphgen.from_edges(n, star + list(zip(a.tolist(), b.tolist())) + bridge)
    G = graph_on_device(g)
    G.set_options(claim_threshold=1 << 30, profile=1)
    for r in (0, 7, 5000):
        say(f"star + random, root {r}")
        assert_bfs_equal(g, G, r)
    info = [L for L in G.level_info() if L["frontier"] > 0]
    assert all(L["mark"] in (0, 3, 4) for L in info)


def test_pull_from_a_few_hubs_below_the_frontier_floor():
    """A frontier of few vertices whose adjacencies times pull_alpha reach
    nnz pulls although it holds fewer vertices than claim_min_frontier (the
    second level of an R-MAT search from a vertex next to the hubs)."""
    g = graphgen.rmat_csr(20, 16, 53)
    G = graph_on_device(g)
    G.set_options(profile=1, claim_min_frontier=16384, pull_alpha=1024)
    seen_small_pull = False
    for r in graphgen.roots(g, 4, 59):
        say(f"rmat20 hub-frontier pull root {r}")
        assert_bfs_equal(g, G, int(r))
        for L in G.level_info():
            if L["mark"] == 2 and 0 < L["frontier"] < 16384:
                assert L["edges"] * 1024 >= g.nnz
                seen_small_pull = True
    assert seen_small_pull
    G.set_options(profile=-1, claim_min_frontier=4096, pull_alpha=14)
