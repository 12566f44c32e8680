"""GPU parity of bfs_run against the CPU oracle, bit for bit (integers)."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import assert_bfs_equal, gpu_bfs, graph_on_device, say, torch_cuda
from paper_1104_4518_amd import bfs as B

pytestmark = pytest.mark.gpu


def test_rmat12_config_all_roots():
    g = graphgen.config_graph("rmat12")
    roots = graphgen.config_roots("rmat12", g)
    G = graph_on_device(g)
    for r in roots:
        say(f"rmat12 root {r}")
        _, ol = assert_bfs_equal(g, G, r)
        st = G.last_stats()
        assert st.edges_traversed == 2 * oracle.reached_edges(g, ol)
        assert st.depth == ol.max()
        assert st.reached == int((ol >= 0).sum())


@pytest.mark.parametrize("name,edges,n", [
    ("path", [(i, i + 1) for i in range(99)], 100),
    ("star", [(0, i) for i in range(1, 300)], 300),
    ("complete", [(i, j) for i in range(40) for j in range(i + 1, 40)], 40),
    ("two_components", [(0, 1), (1, 2), (3, 4), (4, 5), (5, 3)], 8),
    ("single_edge", [(0, 1)], 2),
    ("isolated", [], 5),
])
def test_small_graphs_every_root(name, edges, n):
    g = graphgen.from_edges(n, edges)
    G = graph_on_device(g)
    for r in range(n):
        say(f"{name} root {r}")
        assert_bfs_equal(g, G, r)


def test_claim_level_after_push_level():
    """A claim level that follows a push (mark-and-resolve) level runs before
    that level's resolve writes its vertices' parent words, so its claims
    must still treat those vertices as visited. R-MAT 16 without pull
    levels and with a low vertex floor: the large levels push, the tail
    levels claim."""
    g = graphgen.rmat_csr(16, 16, 23)
    G = graph_on_device(g)
    deg = np.diff(g.off)
    roots = np.random.default_rng(5).choice(np.nonzero(deg > 0)[0], 6, replace=False)
    pairs = 0
    for small in (-1, 8192):
        G.set_options(pull_alpha=-1, claim=3, claim_min_frontier=256, small_frontier=small,
                      profile=1)
        for r in roots:
            say(f"rmat16 push then claim, small_frontier {small}, root {r}")
            assert_bfs_equal(g, G, int(r))
            kinds = [L["mark"] for L in G.level_info() if L["frontier"] > 0]
            pairs += sum(1 for a, b in zip(kinds, kinds[1:]) if a == 1 and b == 0)
    assert pairs > 0


def test_claim_touch_levels_match_oracle():
    """Large claim levels of a symmetric graph claim without touch bytes;
    finish finds their vertices by the level in their parent words. ER
    scale 20 with 2 edges per vertex: its degree-ordered copy's active
    vertices end inside a 32-vertex word (19,098 isolated vertices), and
    with mark levels off the large levels are claim-touch levels."""
    g = graphgen.er_csr(20, 2, 41)
    deg = np.diff(g.off)
    assert (deg == 0).sum() % 32 != 0
    G = graph_on_device(g)
    G.set_options(claim_threshold=1 << 30, pull_alpha=-1, profile=1)
    roots = np.random.default_rng(3).choice(np.nonzero(deg > 0)[0], 3, replace=False)
    kinds = set()
    for r in roots:
        say(f"er20 claim-touch root {r}")
        assert_bfs_equal(g, G, int(r))
        kinds |= {L["mark"] for L in G.level_info() if L["frontier"] > 0}
    assert 3 in kinds


def test_single_vertex():
    g = graphgen.from_edges(1, [])
    G = graph_on_device(g)
    p, lv = gpu_bfs(G, 0)
    assert p.tolist() == [0] and lv.tolist() == [0]


@pytest.mark.parametrize("w", [33, 128])
def test_grid_high_diameter(w):
    g = graphgen.grid_csr(w)
    G = graph_on_device(g)
    for r in (0, w * w // 2 + 3, w * w - 1):
        say(f"grid{w} root {r}")
        assert_bfs_equal(g, G, r)


def test_grid_512_corner():
    g = graphgen.grid_csr(512)
    G = graph_on_device(g)
    say("grid512 root 0")
    _, ol = assert_bfs_equal(g, G, 0)
    assert ol.max() == 1022


@pytest.mark.parametrize("scale,seed", [(14, 21), (16, 22), (18, 23)])
def test_rmat_mid_scales(scale, seed):
    g = graphgen.rmat_csr(scale, 16, seed)
    G = graph_on_device(g)
    for r in graphgen.roots(g, 4, 100 + seed):
        say(f"rmat{scale} root {r}")
        assert_bfs_equal(g, G, r, want_level=(r % 2 == 0))


def test_er_graph():
    g = graphgen.er_csr(16, 16, 7)
    G = graph_on_device(g)
    for r in graphgen.roots(g, 3, 77):
        say(f"er16 root {r}")
        assert_bfs_equal(g, G, r)


def test_directed_csr_follows_stored_adjacencies():
    rng = np.random.default_rng(3)
    n = 3000
    src = rng.integers(0, n, 20000)
    dst = rng.integers(0, n, 20000)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(src, minlength=n))
    g = graphgen.CSR(n, off, dst.astype(np.int32))
    G = graph_on_device(g)
    for r in (0, 17, 2999):
        say(f"directed root {r}")
        assert_bfs_equal(g, G, r)


def test_int32_offsets_and_device_inputs():
    torch = torch_cuda()
    g = graphgen.rmat_csr(12, 16, 9)
    G32 = B.Graph.from_csr(g.n, g.off.astype(np.int32), g.col)
    Gd = B.Graph.from_csr(g.n, torch.from_numpy(g.off).cuda(), torch.from_numpy(g.col).cuda())
    Gd32 = B.Graph.from_csr(g.n, torch.from_numpy(g.off.astype(np.int32)).cuda(),
                            torch.from_numpy(g.col).cuda())
    r = int(graphgen.roots(g, 1, 5)[0])
    for G in (G32, Gd, Gd32):
        say(f"offsets variant root {r}")
        assert_bfs_equal(g, G, r)


def test_host_outputs():
    g = graphgen.rmat_csr(12, 16, 1)
    G = graph_on_device(g)
    r = int(graphgen.roots(g, 1, 1000)[0])
    parent = np.empty(g.n, np.int32)
    level = np.empty(g.n, np.int32)
    say("host outputs")
    G.run(r, parent, level)
    op, ol = oracle.bfs_graph(g, r)
    assert np.array_equal(parent, op) and np.array_equal(level, ol)


def test_stream_argument():
    torch = torch_cuda()
    g = graphgen.rmat_csr(13, 16, 4)
    G = graph_on_device(g)
    s = torch.cuda.Stream()
    r = int(graphgen.roots(g, 1, 44)[0])
    say("explicit stream")
    with torch.cuda.stream(s):
        p, lv = gpu_bfs(G, r, stream=s)
    op, ol = oracle.bfs_graph(g, r)
    assert np.array_equal(p, op) and np.array_equal(lv, ol)


def test_launch_shapes_do_not_change_results():
    """Schedule perturbation: grid sizes, host-check batching and both ways of
    resolving a level's new vertices (atomicMin claims, mark-and-resolve)."""
    g = graphgen.rmat_csr(15, 16, 31)
    G = graph_on_device(g)
    r = int(graphgen.roots(g, 1, 8)[0])
    op, ol = oracle.bfs_graph(g, r)
    for claim in (1, 2, 3):
        for grid, batch in [(1, 1), (3, 2), (17, 16), (256, 1), (4096, 5)]:
            G.set_options(grid_blocks=grid, batch_levels=batch, claim=claim)
            say(f"claim {claim} grid {grid} batch {batch}")
            p, lv = gpu_bfs(G, r, want_level=(grid % 2 == 1))
            assert np.array_equal(p, op), (claim, grid, batch)
            if lv is not None:
                assert np.array_equal(lv, ol), (claim, grid, batch)
            st = G.last_stats()
            if claim == 1:
                assert st.mark_levels == 0
            if claim == 2:
                assert st.mark_levels == st.levels
    for rep in range(5):
        p, lv = gpu_bfs(G, r)
        assert np.array_equal(p, op) and np.array_equal(lv, ol)


def test_symmetry_detection_selects_mark_levels():
    g = graphgen.rmat_csr(16, 16, 12)
    r = int(graphgen.roots(g, 1, 3)[0])
    G = graph_on_device(g)                     # checked at create: symmetric
    say("symmetric detection")
    assert_bfs_equal(g, G, r)
    assert G.last_stats().mark_levels >= 1
    Gt = B.Graph.from_csr(g.n, g.off, g.col, trusted=True)   # unchecked: claims only
    assert_bfs_equal(g, Gt, r)
    assert Gt.last_stats().mark_levels == 0
    Gs = B.Graph.from_csr(g.n, g.off, g.col, trusted=True, symmetric=True)
    assert_bfs_equal(g, Gs, r)
    assert Gs.last_stats().mark_levels >= 1
    # an asymmetric graph is detected and keeps atomicMin claims
    rng = np.random.default_rng(1)
    n = 5000
    src, dst = rng.integers(0, n, 60000), rng.integers(0, n, 60000)
    order = np.lexsort((dst, src))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(src[order], minlength=n))
    gd = graphgen.CSR(n, off, dst[order].astype(np.int32))
    Gd = graph_on_device(gd)
    Gd.set_options(claim=2)
    assert_bfs_equal(gd, Gd, 7)
    assert Gd.last_stats().mark_levels == 0


def test_profile_stats():
    g = graphgen.rmat_csr(14, 16, 2)
    G = graph_on_device(g)
    G.set_options(profile=1)
    r = int(graphgen.roots(g, 1, 2)[0])
    gpu_bfs(G, r)
    st = G.last_stats()
    # launch groups (the device level loop, then one level's kernels): the
    # levels either ran in the loop or each in a group of their own
    lv = G.level_info()
    by_kernels = sum(1 for L in lv if L["frontier"] > 0 and L["mark"] != 4)
    by_loop = sum(1 for L in lv if L["frontier"] > 0 and L["mark"] == 4)
    assert by_loop == st.small_levels and by_kernels + by_loop == st.levels >= 1
    assert st.expand_launches >= by_kernels
    assert st.expand_ms > 0 and st.total_ms >= st.expand_ms + st.small_ms
    assert st.total_ms >= st.finish_ms > 0


def test_errors():
    torch = torch_cuda()
    g = graphgen.rmat_csr(10, 16, 1)
    G = graph_on_device(g)
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(B.BfsError) as ei:
        G.run(g.n, parent)
    assert ei.value.code == B.BFS_ERR_ARG
    with pytest.raises(B.BfsError):
        G.run(-1, parent)
    bad = g.col.copy()
    bad[5] = g.n
    with pytest.raises(B.BfsError) as ei:
        B.Graph.from_csr(g.n, g.off, bad)
    assert ei.value.code == B.BFS_ERR_FORMAT
    off = g.off.copy()
    off[3], off[4] = off[4], off[3] - 1
    with pytest.raises(B.BfsError) as ei:
        B.Graph.from_csr(g.n, off, g.col)
    assert ei.value.code == B.BFS_ERR_FORMAT
    off = g.off.copy()
    off[-1] -= 1
    with pytest.raises(B.BfsError) as ei:
        B.Graph.from_csr(g.n, off, g.col)
    assert ei.value.code == B.BFS_ERR_FORMAT
    # the handle still works after the failed calls
    r = int(graphgen.roots(g, 1, 3)[0])
    assert_bfs_equal(g, G, r)


def test_rmat22_config_sampled_roots():
    """R-MAT scale 22 as benchmarked: full oracle on 3 roots, the definition
    checker on 5 more."""
    g = graphgen.config_graph("rmat22")
    roots = graphgen.config_roots("rmat22", g)
    G = B.Graph.from_csr(g.n, g.off, g.col, trusted=True, symmetric=True)   # as benchmarked
    for r in roots[:3]:
        say(f"rmat22 root {r}")
        assert_bfs_equal(g, G, r)
    for r in roots[3:8]:
        say(f"rmat22 checker root {r}")
        p, lv = gpu_bfs(G, r)
        assert oracle.check_bfs(g, int(r), p, lv) == (0, -1)
    for claim in (1, 2):
        G.set_options(claim=claim)
        say(f"rmat22 claim mode {claim}")
        assert_bfs_equal(g, G, roots[8])


def test_degree_ordered_copy_gives_identical_results():
    """Graphs with n >= 2^20 get a degree-ordered copy for the level kernels;
    outputs stay in the caller's ids and equal the oracle with and without it,
    for both ways of resolving levels and for a directed graph."""
    g = graphgen.rmat_csr(20, 16, 17)
    roots = graphgen.roots(g, 3, 71)
    Gr = B.Graph.from_csr(g.n, g.off, g.col, trusted=True, symmetric=True)
    Gp = B.Graph.from_csr(g.n, g.off, g.col, trusted=True, symmetric=True, relabel=False)
    for r in roots:
        say(f"relabel rmat20 root {r}")
        for claim in (1, 2, 3):
            Gr.set_options(claim=claim)
            Gp.set_options(claim=claim)
            assert_bfs_equal(g, Gr, r, want_level=(claim != 2))
            assert_bfs_equal(g, Gp, r, want_level=(claim != 1))
    rng = np.random.default_rng(5)
    n = 1 << 20
    src, dst = rng.integers(0, n, 3 * n), rng.integers(0, n, 3 * n)
    order = np.lexsort((dst, src))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(src[order], minlength=n))
    gd = graphgen.CSR(n, off, dst[order].astype(np.int32))
    Gd = graph_on_device(gd)
    for r in (0, 12345, n - 1):
        say(f"relabel directed root {r}")
        assert_bfs_equal(gd, Gd, r)


def test_graph_mode_replays_match_oracle():
    """Graph mode (levels captured once in a hipGraph, replayed until the
    frontier is empty): every replay equals the oracle, with eager work and
    synchronisation between runs, new output buffers (a new capture), host
    outputs, a directed graph, both level-resolution ways and a grid deep
    enough for many replays; switching back to level-by-level mode agrees."""
    torch = torch_cuda()
    cases = [("rmat12", graphgen.rmat_csr(12, 16, 1)), ("grid128", graphgen.grid_csr(128)),
             ("rmat16", graphgen.rmat_csr(16, 16, 22))]
    rng = np.random.default_rng(3)
    n = 3000
    src, dst = rng.integers(0, n, 20000), rng.integers(0, n, 20000)
    order = np.lexsort((dst, src))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(src[order], minlength=n))
    cases.append(("directed", graphgen.CSR(n, off, dst[order].astype(np.int32))))
    for name, g in cases:
        G = graph_on_device(g)
        G.set_options(mode=2)
        roots = graphgen.roots(g, 3, 12)
        for claim in (3, 1):
            G.set_options(claim=claim)
            for rep in range(2):
                for r in roots:
                    say(f"graph mode {name} claim {claim} rep {rep} root {r}")
                    assert_bfs_equal(g, G, int(r))
                    # eager work between replays
                    torch.ones(1024, device="cuda").sum().item()
        p = np.empty(g.n, np.int32)
        lv = np.empty(g.n, np.int32)
        say(f"graph mode {name} host outputs")
        G.run(int(roots[0]), p, lv)
        op, ol = oracle.bfs_graph(g, int(roots[0]))
        assert np.array_equal(p, op) and np.array_equal(lv, ol)
        G.set_options(mode=1)
        say(f"level mode {name} after graph mode")
        assert_bfs_equal(g, G, int(roots[1]))


def test_repeated_runs_many_roots_are_exact():
    """Many roots, repeated, under the default policy and with every level
    mark-and-resolve: the frontier order changes from run to run (atomic
    slot reservations), so tiles meet rows in ever new layouts; every run
    must equal the oracle (a lane-shuffle from an inactive lane in a level's
    last, partial tile once turned ~3% of such runs wrong)."""
    g = graphgen.rmat_csr(16, 16, 5)
    rng = np.random.default_rng(7)
    cand = np.nonzero(np.diff(g.off) > 0)[0]
    roots = rng.choice(cand, 40, replace=False)
    ref = {int(r): oracle.bfs_graph(g, int(r)) for r in roots}
    for claim in (3, 2):
        G = graph_on_device(g)
        G.set_options(claim=claim)
        for rep in range(3):
            say(f"repeated runs claim {claim} rep {rep}")
            for r in roots:
                p, lv = gpu_bfs(G, int(r))
                op, ol = ref[int(r)]
                assert np.array_equal(p, op) and np.array_equal(lv, ol), (claim, rep, int(r))


@pytest.mark.parametrize("limit", [-1, 1, 64, 1000, 8192])
def test_device_level_loop_limits_give_identical_results(limit):
    """The device level loop for small frontiers hands levels back to the
    level kernels at different frontier sizes (off, 1, 64, 1000, 8192
    vertices): every setting gives the oracle's arrays."""
    graphs = [graphgen.rmat_csr(16, 16, 41), graphgen.grid_csr(96),
              graphgen.er_csr(15, 4, 42), graphgen.from_edges(6, [(0, 1), (1, 2), (2, 3)])]
    for g in graphs:
        G = graph_on_device(g)
        G.set_options(small_frontier=limit)
        for r in (list(graphgen.roots(g, 3, 43)) if g.n > 6 else [0, 3, 5]):
            say(f"loop limit {limit} n {g.n} root {r}")
            assert_bfs_equal(g, G, int(r))
            st = G.last_stats()
            if limit == -1:
                assert st.small_levels == 0


def test_grid2048_corner_runs_in_the_device_loop():
    """4,094 levels of at most 2,048 vertices, and the level that finds the
    far corner's neighbours all visited: every one runs in the device loop,
    and the level record lists each as a loop level."""
    g = graphgen.grid_csr(2048)
    G = graph_on_device(g)
    G.set_options(profile=1)
    say("grid2048 root 0")
    _, ol = assert_bfs_equal(g, G, 0)
    st = G.last_stats()
    assert ol.max() == 4094 and st.depth == 4094
    assert st.small_levels == st.levels == 4095
    lv = G.level_info()
    assert [L["level"] for L in lv[:3]] == [1, 2, 3]
    assert all(L["mark"] == 4 for L in lv[:4095])
    assert lv[0]["frontier"] == 1 and lv[1]["frontier"] == 2
    G.set_options(profile=-1)
