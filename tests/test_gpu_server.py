"""Continuous-batching server: each result equals the oracle (and so the
query run alone), under admission pressure, step budgets that force queries
to resume across device steps, and host-forced failure paths."""
import time

import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import graph_on_device, say, torch_cuda
from paper_1104_4518_amd import bfs as B

pytestmark = pytest.mark.gpu


def _submit_all(S, items):
    torch = torch_cuda()
    out = []
    for G, r, g in items:
        p = torch.empty(G.n, dtype=torch.int32, device="cuda")
        lv = torch.empty(G.n, dtype=torch.int32, device="cuda")
        out.append((S.submit(G, r, p, lv), p, lv, g, r))
    return out


def _check_all(S, subs):
    for t, p, lv, g, r in subs:
        res = S.wait(t, 120.0)
        assert res.status == B.BFS_OK
        assert res.t_arrive <= res.t_admit <= res.t_done
        op, ol = oracle.bfs_graph(g, r)
        assert np.array_equal(p.cpu().numpy(), op), (g.name, r)
        assert np.array_equal(lv.cpu().numpy(), ol), (g.name, r)
        assert res.depth == ol.max()
        assert res.edges_traversed == int(np.diff(g.off)[ol >= 0].sum())


def test_server_mixed_queries():
    gs = [graphgen.rmat_csr(12, 16, 1), graphgen.grid_csr(128), graphgen.rmat_csr(14, 16, 2)]
    Gs = [graph_on_device(g) for g in gs]
    items = []
    for g, G in zip(gs, Gs):
        for r in graphgen.roots(g, 8, 5):
            items.append((G, int(r), g))
    S = B.Server(slots=16)
    say(f"server {len(items)} queries")
    subs = _submit_all(S, items)
    _check_all(S, subs)
    S.drain()
    S.destroy()
    # the R-MAT graphs above 2^16 adjacencies now take the whole-GPU lane,
    # concurrently with the grid queries in the multi-query steps
    S = B.Server(slots=16, large_query_nnz=1 << 16)
    say(f"server with lane {len(items)} queries")
    subs = _submit_all(S, items)
    _check_all(S, subs)
    S.destroy()


def test_server_admission_by_memory_and_resume():
    """A budget that fits one query's workspace at a time, and a 20 us step
    budget so long queries are suspended and resumed many times (LDS-bitmap
    and global-bitmap graphs)."""
    g_small = graphgen.grid_csr(200)              # bitmap in LDS
    g_big = graphgen.grid_csr(800)                # 640000 vertices: global bitmap
    Gs, Gb = graph_on_device(g_small), graph_on_device(g_big)
    per_query = 2 * ((g_big.n * 4 + 255) // 256 * 256) + (((g_big.n + 31) // 32 * 4 + 255)
                                                          // 256 * 256)
    S = B.Server(slots=8, memory_budget=per_query + 4096, step_budget_us=20)
    items = [(Gs, 0, g_small), (Gb, 5, g_big), (Gs, 199 * 200 + 3, g_small),
             (Gb, 800 * 400 + 400, g_big), (Gs, 777, g_small)]
    say("server admission + resume")
    subs = _submit_all(S, items)
    _check_all(S, subs)
    S.destroy()


def test_server_timeout_busy_and_errors():
    torch = torch_cuda()
    g = graphgen.grid_csr(400)
    G = graph_on_device(g)
    S = B.Server(slots=1)
    say("server timeout/busy")
    subs = _submit_all(S, [(G, i * 997 % g.n, g) for i in range(4)])
    with pytest.raises(B.BfsError) as ei:
        S.wait(subs[-1][0], 0.0001)
    assert ei.value.code == B.BFS_ERR_TIMEOUT
    with pytest.raises(B.BfsError) as ei:
        G.destroy()
    assert ei.value.code == B.BFS_ERR_BUSY
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(B.BfsError) as ei:
        S.submit(G, g.n, p)
    assert ei.value.code == B.BFS_ERR_ARG
    with pytest.raises(B.BfsError) as ei:
        S.submit(G, 0, np.empty(g.n, np.int32))
    assert ei.value.code == B.BFS_ERR_ARG
    _check_all(S, subs)
    S.destroy()
    G.destroy()                                   # no longer busy


def test_server_budget_too_small_rejected():
    g = graphgen.grid_csr(600)     # 2.9 MB of workspace > the 1 MiB budget
    G = graph_on_device(g)
    torch = torch_cuda()
    S = B.Server(slots=2, memory_budget=1 << 20)
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(B.BfsError) as ei:
        S.submit(G, 0, p)
    assert ei.value.code == B.BFS_ERR_CAPACITY
    S.destroy()


def test_server_poisson_arrivals_match_alone():
    """Queries arriving while others run; each result equals its run alone."""
    torch = torch_cuda()
    gs = [graphgen.rmat_csr(13, 16, 3), graphgen.grid_csr(96)]
    Gs = [graph_on_device(g) for g in gs]
    rng = np.random.default_rng(2)
    S = B.Server(slots=32, step_budget_us=100)
    arrivals = graphgen.poisson_arrivals(60, 3000.0, 9)
    subs = []
    t0 = time.perf_counter()
    say("server poisson")
    for a in arrivals:
        while time.perf_counter() - t0 < a:
            pass
        i = int(rng.integers(0, 2))
        g, G = gs[i], Gs[i]
        r = int(rng.integers(0, g.n))
        p = torch.empty(G.n, dtype=torch.int32, device="cuda")
        lv = torch.empty(G.n, dtype=torch.int32, device="cuda")
        subs.append((S.submit(G, r, p, lv), p, lv, g, r))
    _check_all(S, subs)
    S.destroy()
