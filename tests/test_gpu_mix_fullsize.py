"""The batched and served paths on the benchmark mix's full-size graphs
(R-MAT scale 22 of the mix's seed and the 2048 x 2048 grid), element-wise
against the oracle: each query's result is the same alone and in the mix."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import say, torch_cuda
from paper_1104_4518_amd import bfs as B

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _mix_graphs():
    # the two largest graphs of the benchmark mix (same generators and seeds)
    g1 = graphgen.rmat_csr(22, 16, 5)
    g1.name = "rmat22"
    g2 = graphgen.grid_csr(2048)
    g2.name = "grid2048"
    return g1, g2


def _queries(g1, g2, G1, G2):
    rng = np.random.default_rng(1004)
    out = []
    for g, G in ((g1, G1), (g2, G2)):
        cand = np.nonzero(np.diff(g.off) > 0)[0]
        for r in rng.choice(cand, 3, replace=False):
            out.append((G, int(r), g))
    out.append((G2, 0, g2))                 # corner of the grid: 4,094 levels
    return out


def _oracle_cache(items):
    ref = {}
    for _, r, g in items:
        if (g.name, r) not in ref:
            ref[(g.name, r)] = oracle.bfs_graph(g, r)
    return ref


def test_batch_on_mix_fullsize_graphs():
    torch = torch_cuda()
    g1, g2 = _mix_graphs()
    G1 = B.Graph.from_csr(g1.n, g1.off, g1.col, trusted=True, symmetric=True)
    G2 = B.Graph.from_csr(g2.n, g2.off, g2.col, trusted=True, symmetric=True)
    items = _queries(g1, g2, G1, G2)
    ref = _oracle_cache(items)
    ps = [torch.full((G.n,), -5, dtype=torch.int32, device="cuda") for G, _, _ in items]
    ls = [torch.full((G.n,), -5, dtype=torch.int32, device="cuda") for G, _, _ in items]
    say(f"batch of {len(items)} full-size mix queries")
    B.run_batch([G for G, _, _ in items], [r for _, r, _ in items], ps, ls)
    torch.cuda.synchronize()
    for i, (_, r, g) in enumerate(items):
        op, ol = ref[(g.name, r)]
        assert np.array_equal(ps[i].cpu().numpy(), op), (g.name, r)
        assert np.array_equal(ls[i].cpu().numpy(), ol), (g.name, r)


@pytest.mark.parametrize("lane", [0, -1], ids=["lane", "steps_only"])
def test_server_on_mix_fullsize_graphs(lane):
    """With the whole-GPU lane (R-MAT 22 runs there, the grid in the
    multi-query steps) and without it (every query in the steps, resumed
    across many step budgets)."""
    torch = torch_cuda()
    g1, g2 = _mix_graphs()
    G1 = B.Graph.from_csr(g1.n, g1.off, g1.col, trusted=True, symmetric=True)
    G2 = B.Graph.from_csr(g2.n, g2.off, g2.col, trusted=True, symmetric=True)
    items = _queries(g1, g2, G1, G2)
    ref = _oracle_cache(items)
    S = B.Server(slots=8, large_query_nnz=lane)
    subs = []
    say(f"server ({'lane' if lane == 0 else 'steps only'}) {len(items)} full-size queries")
    for G, r, g in items:
        p = torch.full((G.n,), -5, dtype=torch.int32, device="cuda")
        lv = torch.full((G.n,), -5, dtype=torch.int32, device="cuda")
        subs.append((S.submit(G, r, p, lv), p, lv, g, r))
    for t, p, lv, g, r in subs:
        res = S.wait(t, 300.0)
        assert res.status == B.BFS_OK
        op, ol = ref[(g.name, r)]
        assert np.array_equal(p.cpu().numpy(), op), (g.name, r)
        assert np.array_equal(lv.cpu().numpy(), ol), (g.name, r)
        assert res.depth == ol.max()
    S.destroy()
