"""GPU parity of the multi-query path (bfs_run_batch): every query of a mixed
batch must equal the oracle and bfs_run on its own, bit for bit."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import gpu_bfs, graph_on_device, say, torch_cuda
from paper_1104_4518_amd import bfs as B

pytestmark = pytest.mark.gpu


def _directed(n, m, seed):
    rng = np.random.default_rng(seed)
    src, dst = rng.integers(0, n, m), rng.integers(0, n, m)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(src, minlength=n))
    return graphgen.CSR(n, off, dst.astype(np.int32), name="directed")


def _run_batch(pairs, with_levels=True):
    torch = torch_cuda()
    graphs = [G for (G, _, _) in pairs]
    roots = [r for (_, r, _) in pairs]
    parents = [torch.empty(G.n, dtype=torch.int32, device="cuda") for G in graphs]
    levels = [torch.empty(G.n, dtype=torch.int32, device="cuda") if with_levels or i % 2 else None
              for i, G in enumerate(graphs)]
    B.run_batch(graphs, roots, parents, levels)
    torch.cuda.synchronize()
    return parents, levels


def test_mixed_batch_matches_oracle_and_plain():
    specs = [graphgen.rmat_csr(10, 16, 1), graphgen.rmat_csr(12, 16, 2),
             graphgen.rmat_csr(14, 16, 3), graphgen.grid_csr(64), graphgen.grid_csr(16, 5),
             graphgen.er_csr(11, 8, 4), _directed(2000, 9000, 5),
             graphgen.from_edges(7, [(0, 1), (1, 2), (4, 5)])]
    devs = [graph_on_device(g) for g in specs]
    pairs = []
    for g, G in zip(specs, devs):
        rs = graphgen.roots(g, 5, 17) if g.nnz else np.array([0], np.int32)
        if g.n == 7:
            rs = np.array([0, 3, 6], np.int32)      # isolated roots too
        for r in rs:
            pairs.append((G, int(r), g))
    say(f"batch of {len(pairs)} queries")
    parents, levels = _run_batch(pairs)
    for i, (G, r, g) in enumerate(pairs):
        op, ol = oracle.bfs_graph(g, r)
        assert np.array_equal(parents[i].cpu().numpy(), op), (g.name, r)
        assert np.array_equal(levels[i].cpu().numpy(), ol), (g.name, r)
    # the same queries alone through bfs_run
    for i, (G, r, g) in enumerate(pairs[::7]):
        p, lv = gpu_bfs(G, r)
        op, ol = oracle.bfs_graph(g, r)
        assert np.array_equal(p, op) and np.array_equal(lv, ol)


def test_batch_large_graph_global_bitmap():
    """Graphs above the LDS bitmap capacity use the workspace bitmap."""
    g1 = graphgen.rmat_csr(20, 16, 8)
    g2 = graphgen.grid_csr(1024)
    G1, G2 = graph_on_device(g1), graph_on_device(g2)
    pairs = [(G1, int(r), g1) for r in graphgen.roots(g1, 3, 9)]
    pairs += [(G2, 0, g2), (G2, 1024 * 512 + 77, g2)]
    say("batch with large graphs")
    parents, levels = _run_batch(pairs, with_levels=False)
    for i, (G, r, g) in enumerate(pairs):
        op, ol = oracle.bfs_graph(g, r)
        assert np.array_equal(parents[i].cpu().numpy(), op)
        if levels[i] is not None:
            assert np.array_equal(levels[i].cpu().numpy(), ol)


def test_batch_many_small_queries():
    g = graphgen.rmat_csr(13, 16, 6)
    G = graph_on_device(g)
    roots = graphgen.roots(g, 600, 61)
    pairs = [(G, int(r), g) for r in roots]
    say(f"batch of {len(pairs)} small queries")
    parents, levels = _run_batch(pairs)
    for i in range(0, len(pairs), 37):
        op, ol = oracle.bfs_graph(g, pairs[i][1])
        assert np.array_equal(parents[i].cpu().numpy(), op)
        assert np.array_equal(levels[i].cpu().numpy(), ol)


def test_batch_argument_errors():
    torch = torch_cuda()
    g = graphgen.rmat_csr(10, 16, 1)
    G = graph_on_device(g)
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    q = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(B.BfsError) as ei:
        B.run_batch([G, G], [0, 1], [p, p])               # aliasing outputs
    assert ei.value.code == B.BFS_ERR_ARG
    with pytest.raises(B.BfsError) as ei:
        B.run_batch([G], [g.n], [p])                      # root out of range
    assert ei.value.code == B.BFS_ERR_ARG
    with pytest.raises(B.BfsError) as ei:
        B.run_batch([G], [0], [np.empty(g.n, np.int32)])  # host output
    assert ei.value.code == B.BFS_ERR_ARG
    B.run_batch([], [], [])                               # empty batch is fine
    B.run_batch([G, G], [0, 5], [p, q])
    torch.cuda.synchronize()
    op, _ = oracle.bfs_graph(g, 5)
    assert np.array_equal(q.cpu().numpy(), op)
