"""Symmetric (upper-triangle) storage, BFS_UPPER: the library holds each
undirected edge once, in the row of its smaller endpoint, and searches the
symmetric closure. Levels and parents must equal the oracle's on the full
graph, bit for bit."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import gpu_bfs, say, torch_cuda
from paper_1104_4518_amd import bfs as B

pytestmark = pytest.mark.gpu


def upper_on_device(g, **kw):
    u = graphgen.upper_csr(g)
    return B.Graph.from_csr(u.n, u.off, u.col, upper=True, **kw)


def check(g, G, root):
    p, lv = gpu_bfs(G, root)
    op, ol = oracle.bfs_graph(g, int(root))
    assert np.array_equal(lv, ol), f"level mismatch at root {root}"
    assert np.array_equal(p, op), f"parent mismatch at root {root}: {np.nonzero(p != op)[0][:8]}"
    st = G.last_stats()
    assert st.reached == int((ol >= 0).sum())
    assert st.depth == int(ol.max())
    return ol


@pytest.mark.parametrize("name,edges,n", [
    ("path", [(i, i + 1) for i in range(99)], 100),
    ("reversed_path", [(i, i + 1) for i in range(60)], 61),
    ("star", [(0, i) for i in range(1, 300)], 300),
    ("star_last_centre", [(i, 299) for i in range(299)], 300),
    ("complete", [(i, j) for i in range(40) for j in range(i + 1, 40)], 40),
    ("cycle", [(i, (i + 1) % 50) for i in range(50)], 50),
    ("two_components", [(0, 1), (1, 2), (3, 4), (4, 5), (5, 3)], 8),
    ("isolated", [], 5),
])
def test_closed_forms_every_root(name, edges, n):
    g = graphgen.from_edges(n, edges)
    G = upper_on_device(g)
    for r in range(n):
        say(f"upper {name} root {r}")
        check(g, G, r)


@pytest.mark.parametrize("w", [33, 128])
def test_grids(w):
    g = graphgen.grid_csr(w)
    G = upper_on_device(g)
    for r in (0, w * w // 2 + 3, w * w - 1):
        say(f"upper grid{w} root {r}")
        ol = check(g, G, r)
        i, j = divmod(r, w)
        ii, jj = np.divmod(np.arange(w * w), w)
        assert np.array_equal(ol, np.abs(ii - i) + np.abs(jj - j))


@pytest.mark.parametrize("kind,scale,seed", [("rmat", 14, 31), ("rmat", 18, 32), ("er", 16, 33)])
def test_random_graphs(kind, scale, seed):
    g = graphgen.rmat_csr(scale, 16, seed) if kind == "rmat" else graphgen.er_csr(scale, 16, seed)
    G = upper_on_device(g)
    for r in graphgen.roots(g, 4, 200 + seed):
        say(f"upper {kind}{scale} root {r}")
        check(g, G, int(r))


def test_rmat22_config_roots_and_handle_reuse():
    g = graphgen.config_graph("rmat22")
    roots = graphgen.config_roots("rmat22", g)
    G = upper_on_device(g, trusted=True)
    _, nnz, dev_bytes = G.info()
    assert nnz * 2 == g.nnz
    for r in roots[:3]:
        say(f"upper rmat22 root {r}")
        check(g, G, int(r))


def test_upper_input_is_validated():
    # an adjacency below its row, and a row out of order
    with pytest.raises(B.BfsError) as ei:
        B.Graph.from_csr(3, np.array([0, 1, 2, 2]), np.array([1, 0], np.int32), upper=True)
    assert ei.value.code == B.BFS_ERR_FORMAT
    with pytest.raises(B.BfsError) as ei:
        B.Graph.from_csr(4, np.array([0, 2, 2, 2, 2]), np.array([3, 2], np.int32), upper=True)
    assert ei.value.code == B.BFS_ERR_FORMAT


def test_batch_rejects_upper_graphs_and_server_lane_runs_them():
    torch = torch_cuda()
    g = graphgen.rmat_csr(12, 16, 9)
    G = upper_on_device(g)
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    r = int(graphgen.roots(g, 1, 4)[0])
    with pytest.raises(B.BfsError) as ei:
        B.run_batch([G], [r], [p], [lv])
    assert ei.value.code == B.BFS_ERR_UNSUPPORTED
    say("upper graph through the server")
    S = B.Server(slots=4)
    t = S.submit(G, r, p, lv)
    S.drain()
    assert S.poll(t).status == B.BFS_OK
    S.destroy()
    torch.cuda.synchronize()
    op, ol = oracle.bfs_graph(g, r)
    assert np.array_equal(p.cpu().numpy(), op) and np.array_equal(lv.cpu().numpy(), ol)
